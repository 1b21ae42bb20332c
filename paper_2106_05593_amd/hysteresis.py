"""Adaptive hysteresis-loop driver (paper Sec. III, hysteresis loops).

At every field step the chain runs chunks of `chunk` sweeps and averages m
along the field direction over each chunk (from the per-sweep FP64 means the
library records).  The step is done once at least `min_chunks` chunks have
run and the last two chunk averages differ by less than `tol` (in units of
Ms0); the last chunk average is the loop point, and the next field starts from
the state the chain is in.  As in the paper only the increasing branch is
simulated; the decreasing branch follows by inverse symmetry,
m_dec(H) = -m_inc(-H).

The driver is host logic around any object with `set_field(B_tesla[3])` and
`sweep_record(n) -> (n, 5) array` whose first three columns are <mx>, <my>,
<mz> after each sweep (`Chain` is one).

`hysteresis_loops` runs several independent loops (chains at different
temperatures, seeds or materials) as one batch: every chunk is one batched
launch of all chains, and each chain's chunk average comes from the library's
on-device running averages (`take_averages`).  Each chain applies the rule
above on its own; a chain whose step has converged keeps sweeping at its field
until every chain's step has, and its loop point is the chunk average at its
own convergence.

Each loop point of the single-chain driver carries the standard error of its
chunk average, estimated from the chunk's per-sweep series by blocking
(Flyvbjerg and Petersen, J. Chem. Phys. 91, 461 (1989)): successive halvings of
the series into block means, the largest naive error over the levels that
keep at least `min_blocks` blocks, which bounds the error of correlated samples
once the blocks are longer than the correlation time.
"""
import numpy as np


def blocked_se(x, min_blocks=16):
    """Standard error of the mean of a correlated series by blocking (the
    maximum over blocking levels with at least min_blocks blocks)."""
    x = np.asarray(x, dtype=np.float64).ravel()
    if x.size < 2:
        return float("nan")
    best = 0.0
    while x.size >= max(2, min_blocks):
        best = max(best, float(x.std(ddof=1)) / np.sqrt(x.size))
        h = x.size // 2
        x = 0.5 * (x[0:2 * h:2] + x[1:2 * h:2])
    return best


def field_step(chain, B, direction, chunk=2000, min_chunks=2, tol=0.01, max_chunks=50):
    """Run one field step; returns (loop point, chunks run, converged, standard
    error of the loop point)."""
    if chunk < 1 or min_chunks < 2 or max_chunks < min_chunks or not tol > 0:
        raise ValueError("need chunk >= 1, 2 <= min_chunks <= max_chunks, tol > 0")
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    chain.set_field(tuple(float(B) * d))
    prev = None
    for k in range(1, max_chunks + 1):
        series = np.asarray(chain.sweep_record(chunk))
        along = series[:, :3] @ d
        avg = float(along.mean())
        if k >= min_chunks and abs(avg - prev) < tol:
            return avg, k, True, blocked_se(along)
        prev = avg
    return avg, max_chunks, False, blocked_se(along)


def hysteresis_loop(chain, fields, direction=(0.0, 0.0, 1.0), chunk=2000, min_chunks=2, tol=0.01, max_chunks=50):
    """Increasing-field branch at `fields` (tesla along `direction`, increasing),
    completed by inverse symmetry.  Returns a dict of arrays: H_inc, m_inc,
    m_se (standard error of each point), chunks, converged, and the decreasing
    branch H_dec, m_dec."""
    H = np.asarray(fields, dtype=np.float64)
    if H.ndim != 1 or H.size < 1 or np.any(np.diff(H) <= 0):
        raise ValueError("fields must be a non-empty increasing sequence")
    m = np.zeros(H.size)
    se = np.zeros(H.size)
    chunks = np.zeros(H.size, dtype=np.int64)
    conv = np.zeros(H.size, dtype=bool)
    for i, B in enumerate(H):
        m[i], chunks[i], conv[i], se[i] = field_step(chain, B, direction, chunk, min_chunks, tol, max_chunks)
    return {"H_inc": H, "m_inc": m, "m_se": se, "chunks": chunks, "converged": conv,
            "H_dec": -H, "m_dec": -m}


def hysteresis_loops(batch, chains, fields, direction=(0.0, 0.0, 1.0), chunk=2000, min_chunks=2, tol=0.01,
                     max_chunks=50):
    """Increasing-field branches of several chains advanced together by `batch`
    (an object with `sweep(n)` and `sync()` over `chains`, each with
    `set_field` and `take_averages() -> (avg[4], n)`).  Returns one dict per
    chain, as hysteresis_loop does."""
    H = np.asarray(fields, dtype=np.float64)
    if H.ndim != 1 or H.size < 1 or np.any(np.diff(H) <= 0):
        raise ValueError("fields must be a non-empty increasing sequence")
    if chunk < 1 or min_chunks < 2 or max_chunks < min_chunks or not tol > 0:
        raise ValueError("need chunk >= 1, 2 <= min_chunks <= max_chunks, tol > 0")
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    nc = len(chains)
    m = np.zeros((nc, H.size))
    chunks = np.zeros((nc, H.size), dtype=np.int64)
    conv = np.zeros((nc, H.size), dtype=bool)
    for i, B in enumerate(H):
        for c in chains:
            c.set_field(tuple(float(B) * d))
        batch.sync()
        for c in chains:
            c.take_averages()                       # drop the sums of earlier sweeps
        prev = np.full(nc, np.nan)
        done = np.zeros(nc, dtype=bool)
        for k in range(1, max_chunks + 1):
            batch.sweep(chunk)
            batch.sync()
            for j, c in enumerate(chains):
                avg, n = c.take_averages()
                if done[j]:
                    continue
                a = float(avg[:3] @ d)
                m[j, i], chunks[j, i] = a, k
                if k >= min_chunks and abs(a - prev[j]) < tol:
                    done[j] = conv[j, i] = True
                prev[j] = a
            if done.all():
                break
    return [{"H_inc": H, "m_inc": m[j], "chunks": chunks[j], "converged": conv[j], "H_dec": -H, "m_dec": -m[j]}
            for j in range(nc)]
