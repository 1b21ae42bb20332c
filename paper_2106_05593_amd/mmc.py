"""Thin ctypes binding of libmmc (include/mmc.h).

Argument marshalling only: every step of the Monte Carlo path runs in the HIP
library.  The binding refuses to work without the built library (there is no
CPU fallback).  PyTorch is used only to hand device memory and the current HIP
stream to the library.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libmmc.so")

MMC_OK, MMC_ERR_ARG, MMC_ERR_DOMAIN, MMC_ERR_OOM, MMC_ERR_DEVICE, MMC_ERR_STATE, MMC_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
MMC_MF_LANGEVIN, MMC_MF_BRILLOUIN_HALF = 0, 1
MMC_LEN_PAPER, MMC_LEN_EXACT = 0, 1
MMC_DEMAG_OFF, MMC_DEMAG_FP32, MMC_DEMAG_SPLIT_BF16, MMC_DEMAG_SPLIT_FP16 = 0, 1, 2, 3
_DEMAG_MODES = {False: MMC_DEMAG_OFF, True: MMC_DEMAG_FP32, "off": MMC_DEMAG_OFF, "fp32": MMC_DEMAG_FP32,
                "split_bf16": MMC_DEMAG_SPLIT_BF16, "split_fp16": MMC_DEMAG_SPLIT_FP16}
MMC_ANIS_UNIAXIAL, MMC_ANIS_CUBIC = 0, 1
MMC_SCHED_AUTO, MMC_SCHED_GROUPS, MMC_SCHED_PERSISTENT = 0, 1, 2
_SCHEDS = {"auto": MMC_SCHED_AUTO, "groups": MMC_SCHED_GROUPS, "persistent": MMC_SCHED_PERSISTENT}
MUB = 9.2740100783e-24


class MMCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (status %d)" % (msg, status))
        self.status = status


class mmc_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32)]


class mmc_cellsize(C.Structure):
    _fields_ = [("hx", C.c_double), ("hy", C.c_double), ("hz", C.c_double)]


class mmc_material(C.Structure):
    _fields_ = [("Ms0", C.c_double), ("A0", C.c_double), ("D0", C.c_double), ("K1", C.c_double),
                ("K2", C.c_double), ("easy_axis", C.c_double * 3), ("Tc", C.c_double),
                ("mu_atomic", C.c_double), ("mf", C.c_int32)]


class mmc_run(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("chain_id", C.c_uint32), ("cone_deg", C.c_int32),
                ("adapt_every", C.c_int32), ("sigma_fixed", C.c_double), ("lenmove", C.c_int32),
                ("demag", C.c_int32), ("refresh_per_sweep", C.c_int32), ("T", C.c_double),
                ("B", C.c_double * 3), ("init", C.c_int32), ("init_dir", C.c_double * 3)]


class mmc_stats(C.Structure):
    _fields_ = [("sweeps", C.c_uint64), ("accepts_window", C.c_uint64), ("cone_deg", C.c_int32),
                ("sigma", C.c_double), ("me", C.c_double), ("m_mean", C.c_double * 3),
                ("m2_mean", C.c_double), ("accepts_last", C.c_uint64)]


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "mmc_create": (C.c_int, [C.POINTER(mmc_grid), C.POINTER(mmc_cellsize), C.POINTER(mmc_material),
                             C.POINTER(mmc_run), C.c_void_p, C.POINTER(C.c_void_p)]),
    "mmc_destroy": (None, [C.c_void_p]),
    "mmc_set_grains": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_double]),
    "mmc_set_field": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "mmc_set_temperature": (C.c_int, [C.c_void_p, C.c_double]),
    "mmc_set_grain_temperatures": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32]),
    "mmc_set_anisotropy": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32,
                                     C.c_int32]),
    "mmc_set_m": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "mmc_get_m": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "mmc_sweep": (C.c_int, [C.c_void_p, C.c_int32]),
    "mmc_sweep_record": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "mmc_sweep_timed": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    "mmc_energy": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "mmc_energy_noalloc": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mmc_demag_field": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "mmc_subsweep": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "mmc_get_stats": (C.c_int, [C.c_void_p, C.POINTER(mmc_stats)]),
    "mmc_get_tuning": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mmc_take_averages": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]),
    "mmc_get_state": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_int32), C.POINTER(C.c_uint64)]),
    "mmc_set_state": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int32, C.c_uint64]),
    "mmc_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p)]),
    "mmc_batch_sweep": (C.c_int, [C.c_void_p, C.c_int32]),
    "mmc_batch_sync": (C.c_int, [C.c_void_p]),
    "mmc_batch_destroy": (None, [C.c_void_p]),
    "mmc_batch_set_schedule": (C.c_int, [C.c_void_p, C.c_int32]),
    "mmc_batch_get_schedule": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.c_void_p]),
    "mmc_sync": (C.c_int, [C.c_void_p]),
    "mmc_status_str": (C.c_char_p, [C.c_int]),
    "mmc_last_error": (C.c_char_p, []),
}
EXPORTS = tuple(_SIGS)


def lib():
    """Load libmmc.so (built by paper_2106_05593_amd/build.py); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            raise ImportError("libmmc.so is not built: run python -c 'import __graft_entry__ as g; g.build()'")
        L = C.CDLL(SO)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != MMC_OK:
        raise MMCError(status, lib().mmc_last_error().decode())


def _current_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


class Chain:
    """One Markov chain on the GPU (a context of libmmc).

    grid (nx, ny, nz), cell (hx, hy, hz) in m; material constants in SI; T in K;
    B = mu0*H in tesla.  stream: 'torch' (torch's current stream), None (a
    library-owned stream) or an integer hipStream_t.
    """

    def __init__(self, grid, cell, Ms0, A0, K1, Tc, T, D0=0.0, K2=0.0, easy_axis=(0, 0, 1), B=(0, 0, 0),
                 mf=MMC_MF_BRILLOUIN_HALF, mu=MUB, seed=0, chain_id=0, cone_deg=30, adapt_every=100,
                 sigma_fixed=0.0, lenmove=MMC_LEN_PAPER, demag=False, refresh_per_sweep=2, init=0,
                 init_dir=(0, 0, 1), stream=None):
        self.grid = tuple(int(v) for v in grid)
        self.N = int(np.prod(self.grid))
        g = mmc_grid(*self.grid)
        cs = mmc_cellsize(*[float(v) for v in cell])
        mat = mmc_material(Ms0=float(Ms0), A0=float(A0), D0=float(D0), K1=float(K1), K2=float(K2),
                           easy_axis=(C.c_double * 3)(*[float(v) for v in easy_axis]), Tc=float(Tc),
                           mu_atomic=float(mu), mf=int(mf))
        run = mmc_run(seed=int(seed), chain_id=int(chain_id), cone_deg=int(cone_deg), adapt_every=int(adapt_every),
                      sigma_fixed=float(sigma_fixed), lenmove=int(lenmove),
                      demag=_DEMAG_MODES[demag], refresh_per_sweep=int(refresh_per_sweep),
                      T=float(T), B=(C.c_double * 3)(*[float(v) for v in B]), init=int(init),
                      init_dir=(C.c_double * 3)(*[float(v) for v in init_dir]))
        if stream == "torch":
            s = _current_stream()
        elif stream is None:
            s = C.c_void_p(None)
        else:
            s = C.c_void_p(int(stream))
        h = C.c_void_p()
        _check(lib().mmc_create(C.byref(g), C.byref(cs), C.byref(mat), C.byref(run), s, C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().mmc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def set_grains(self, grain_of_cell, easy_axes, K1, K2, Tc, boundary_exchange_scale):
        """Per-cell grain ids (N, natural order) and per-grain easy axis (n, 3),
        K1, K2, Tc (n,); returns the anisotropy to the uniaxial form and clears
        grain temperatures."""
        gid = np.ascontiguousarray(grain_of_cell, dtype=np.uint32).reshape(-1)
        ea = np.ascontiguousarray(easy_axes, dtype=np.float64).reshape(-1)
        k1 = np.ascontiguousarray(K1, dtype=np.float64).reshape(-1)
        k2 = np.ascontiguousarray(K2, dtype=np.float64).reshape(-1)
        tc = np.ascontiguousarray(Tc, dtype=np.float64).reshape(-1)
        n = tc.size
        if gid.size != self.N or ea.size != 3 * n or k1.size != n or k2.size != n:
            raise ValueError("need N grain ids and n easy axes (n, 3), K1, K2, Tc (n,)")
        _check(lib().mmc_set_grains(self._h, gid.ctypes.data, len(tc), ea.ctypes.data, k1.ctypes.data,
                                    k2.ctypes.data, tc.ctypes.data, float(boundary_exchange_scale)))

    def set_field(self, B):
        _check(lib().mmc_set_field(self._h, (C.c_double * 3)(*[float(v) for v in B])))

    def set_temperature(self, T):
        _check(lib().mmc_set_temperature(self._h, float(T)))

    def set_grain_temperatures(self, T_of_grain):
        """Per-grain temperatures (K) of a non-uniform temperature profile, or None."""
        if T_of_grain is None:
            _check(lib().mmc_set_grain_temperatures(self._h, None, 0))
            return
        t = np.ascontiguousarray(T_of_grain, dtype=np.float64)
        _check(lib().mmc_set_grain_temperatures(self._h, t.ctypes.data, int(t.size)))

    def take_averages(self):
        """(averages of <mx>, <my>, <mz>, <|m|^2> over the sweeps since the last
        call, number of those sweeps); resets the device accumulators."""
        avg = (C.c_double * 4)()
        n = C.c_uint64()
        _check(lib().mmc_take_averages(self._h, avg, C.byref(n)))
        return np.array(avg[:]), int(n.value)

    def set_anisotropy(self, kind="uniaxial", axes=None, K1=None, K2=None, me_scaling=False):
        """Anisotropy form: "uniaxial" (material / grain constants) or "cubic" with
        axes (n, 2, 3) first and second crystal axes (or (2, 3) for every cell),
        K1, K2 (n,) cubic constants in J/m^3; me_scaling: me^{l(l+1)/2} law."""
        if kind == "uniaxial":
            _check(lib().mmc_set_anisotropy(self._h, MMC_ANIS_UNIAXIAL, None, None, None, 0, int(bool(me_scaling))))
            return
        if kind != "cubic":
            raise ValueError("kind must be 'uniaxial' or 'cubic'")
        ax = np.ascontiguousarray(axes, dtype=np.float64)
        if ax.size % 6 != 0 or ax.shape[-2:] != (2, 3):
            raise ValueError("axes must be (2, 3) or (n, 2, 3)")
        ax = ax.reshape(-1, 6)
        n = ax.shape[0]
        k1 = np.ascontiguousarray(np.broadcast_to(np.asarray(K1, dtype=np.float64), (n,)))
        k2 = np.ascontiguousarray(np.broadcast_to(np.asarray(K2, dtype=np.float64), (n,)))
        _check(lib().mmc_set_anisotropy(self._h, MMC_ANIS_CUBIC, ax.ctypes.data, k1.ctypes.data, k2.ctypes.data, n,
                                        int(bool(me_scaling))))

    def set_m(self, m):
        """m: numpy (3, N) float32 (host) or torch CUDA tensor (3, N) float32 (device)."""
        if hasattr(m, "is_cuda") and m.is_cuda:
            assert m.dtype.__str__() == "torch.float32" and m.is_contiguous() and m.numel() == 3 * self.N
            _check(lib().mmc_set_m(self._h, _dptr(m), 1))
        else:
            a = np.ascontiguousarray(m, dtype=np.float32).reshape(3, self.N)
            _check(lib().mmc_set_m(self._h, a.ctypes.data, 0))

    def get_m(self, out=None):
        if out is not None:
            assert out.is_cuda and out.is_contiguous() and out.numel() == 3 * self.N
            _check(lib().mmc_get_m(self._h, _dptr(out), 1))
            return out
        a = np.empty((3, self.N), dtype=np.float32)
        _check(lib().mmc_get_m(self._h, a.ctypes.data, 0))
        return a

    def sweep(self, n):
        _check(lib().mmc_sweep(self._h, int(n)))

    def sweep_record(self, n):
        s = np.zeros((int(n), 5))
        _check(lib().mmc_sweep_record(self._h, int(n), s.ctypes.data))
        return s

    def sweep_timed(self, n, every=1):
        """n sweeps with per-kernel HIP-event timing of sweeps 0, every, ...:
        (ms[6], launches[6]) summed over the sampled sweeps, for demag
        x-forward, demag y-pass, demag x-inverse, colour pass, end of sweep,
        fused colour pass (x-inverse, pass, x-forward)."""
        ms = np.zeros(6)
        cnt = np.zeros(6, dtype=np.int32)
        _check(lib().mmc_sweep_timed(self._h, int(n), int(every), ms.ctypes.data, cnt.ctypes.data))
        return ms, cnt

    def energy(self):
        tot = C.c_double()
        terms = (C.c_double * 6)()
        _check(lib().mmc_energy(self._h, C.byref(tot), terms))
        return tot.value, np.array(terms[:])

    def energy_noalloc(self, out):
        """mmc_energy_noalloc: enqueue the energy into out (torch CUDA float64
        tensor of 7 elements: six terms, then the total); no allocation, no sync."""
        if out.dtype != np.float64 and str(out.dtype) != "torch.float64":
            raise TypeError("out must be float64")
        if not out.is_cuda or out.numel() < 7 or not out.is_contiguous():
            raise ValueError("out must be a contiguous CUDA tensor of at least 7 elements")
        _check(lib().mmc_energy_noalloc(self._h, _dptr(out)))

    def demag_field(self):
        a = np.empty((3, self.N), dtype=np.float32)
        _check(lib().mmc_demag_field(self._h, a.ctypes.data, 0))
        return a

    def subsweep(self, colour, h=None):
        """One colour pass with frozen field h (torch CUDA (3,N) float32 or None);
        returns the per-cell decisions as a torch uint8 CUDA tensor."""
        import torch
        acc = torch.empty(self.N, dtype=torch.uint8, device="cuda")
        hp = _dptr(h) if h is not None else C.c_void_p(None)
        _check(lib().mmc_subsweep(self._h, int(colour), hp, _dptr(acc)))
        return acc

    def stats(self):
        s = mmc_stats()
        _check(lib().mmc_get_stats(self._h, C.byref(s)))
        return {"sweeps": s.sweeps, "accepts_window": s.accepts_window, "cone_deg": s.cone_deg, "sigma": s.sigma,
                "me": s.me, "m_mean": list(s.m_mean), "m2_mean": s.m2_mean, "accepts_last": s.accepts_last}

    def tuning(self):
        """(rows per thread of the x passes (forward, inverse), us per launch of
        the candidates 1, 2, 4 for each direction, colour-pass form (0 separate,
        1 fused, 2 half fused), us per colour of forms 0, 1, 2)."""
        rpt = np.zeros(2, dtype=np.int32)
        us = np.zeros(6)
        fz = C.c_int32()
        fus = np.zeros(3)
        _check(lib().mmc_get_tuning(self._h, rpt.ctypes.data, us.ctypes.data, C.byref(fz), fus.ctypes.data))
        return tuple(int(v) for v in rpt), us, int(fz.value), fus

    def get_state(self):
        sw, cd, win = C.c_uint64(), C.c_int32(), C.c_uint64()
        _check(lib().mmc_get_state(self._h, C.byref(sw), C.byref(cd), C.byref(win)))
        return sw.value, cd.value, win.value

    def set_state(self, sweep, cone_deg, window):
        _check(lib().mmc_set_state(self._h, int(sweep), int(cone_deg), int(window)))

    def sync(self):
        _check(lib().mmc_sync(self._h))


class Batch:
    """Independent chains advanced together by one HIP graph launch per call.

    schedule: 'auto' (timed choice), 'groups' (shape groups sharing launches)
    or 'persistent' (one persistent kernel for every chain)."""

    def __init__(self, chains, schedule="auto"):
        self.chains = list(chains)
        arr = (C.c_void_p * len(self.chains))(*[c.handle.value for c in self.chains])
        h = C.c_void_p()
        _check(lib().mmc_batch_create(arr, len(self.chains), C.byref(h)))
        self._h = h
        if schedule != "auto":
            self.set_schedule(schedule)

    def set_schedule(self, schedule):
        _check(lib().mmc_batch_set_schedule(self._h, _SCHEDS[schedule]))

    def schedule(self):
        """(form in use: 'groups' or 'persistent', trial ms of (groups, persistent))."""
        used = C.c_int32()
        ms = np.zeros(2)
        _check(lib().mmc_batch_get_schedule(self._h, C.byref(used), ms.ctypes.data))
        return {v: k for k, v in _SCHEDS.items()}[used.value], ms

    def sweep(self, n):
        _check(lib().mmc_batch_sweep(self._h, int(n)))

    def sync(self):
        _check(lib().mmc_batch_sync(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().mmc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
