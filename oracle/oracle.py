"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It loads oracle/libmmc_oracle.so (plain C, built by
oracle/build_oracle.py) and never touches the GPU library.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(HERE, "libmmc_oracle.so")
_lib = None

KB = 1.380649e-23
MUB = 9.2740100783e-24
MU0 = 4e-7 * np.pi


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            from . import build_oracle  # noqa: WPS433
            build_oracle.build()
        _lib = C.CDLL(_SO)
        _declare(_lib)
    return _lib


class OrClass(C.Structure):
    _fields_ = [("me", C.c_double), ("inv_chi", C.c_double), ("below", C.c_int),
                ("la", C.c_double), ("lb", C.c_double), ("lbc", C.c_double),
                ("sigma", C.c_double), ("m0", C.c_double)]


class OrSys(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("hx", C.c_double), ("hy", C.c_double), ("hz", C.c_double),
                ("Ms0", C.c_double), ("A0", C.c_double), ("D0", C.c_double),
                ("T", C.c_double), ("B", C.c_double * 3), ("mf", C.c_int32), ("mu", C.c_double),
                ("lenmode", C.c_int32), ("demag", C.c_int32), ("refresh_per_sweep", C.c_int32),
                ("seed", C.c_uint64), ("chain_id", C.c_uint32), ("sigma_fixed", C.c_double),
                ("nclass", C.c_int32), ("cls", C.POINTER(C.c_uint32)), ("ea", C.POINTER(C.c_double)),
                ("K1", C.POINTER(C.c_double)), ("K2", C.POINTER(C.c_double)), ("Tc", C.POINTER(C.c_double)),
                ("bscale", C.c_double), ("Tcl", C.POINTER(C.c_double)),
                ("anis", C.c_int32), ("cax", C.POINTER(C.c_double)), ("kscale", C.c_int32)]


_dp = C.POINTER(C.c_double)


def _declare(L):
    L.or_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
    L.or_u01.argtypes = [C.c_uint32]
    L.or_u01.restype = C.c_double
    L.or_meanfield.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, _dp, _dp]
    L.or_class_coeffs.argtypes = [C.POINTER(OrSys), C.POINTER(OrClass)]
    for nm in ("or_newell", "or_newell_exact"):
        getattr(L, nm).argtypes = [C.c_double] * 6 + [_dp]
    L.or_newell_far.argtypes = [C.c_double] * 6 + [C.c_int, _dp]
    L.or_dinvr.argtypes = [C.c_int] * 3 + [C.c_double] * 3
    L.or_dinvr.restype = C.c_double
    L.or_demag_direct.argtypes = [C.c_int] * 3 + [C.c_double] * 3 + [_dp, _dp]
    L.or_demag_direct_at.argtypes = [C.c_int] * 3 + [C.c_double] * 3 + [_dp, C.POINTER(C.c_int64), C.c_int, _dp]
    L.or_demag_plan_create.argtypes = [C.c_int] * 3 + [C.c_double] * 3
    L.or_demag_plan_create.restype = C.c_void_p
    L.or_demag_plan_apply.argtypes = [C.c_void_p, _dp, _dp]
    L.or_demag_plan_destroy.argtypes = [C.c_void_p]
    L.or_delta_F.argtypes = [C.POINTER(OrSys), C.POINTER(OrClass), _dp, _dp, C.c_int64, _dp, _dp]
    L.or_energy.argtypes = [C.POINTER(OrSys), C.POINTER(OrClass), _dp, _dp, _dp]
    L.or_subsweep.argtypes = [C.POINTER(OrSys), C.POINTER(OrClass), _dp, _dp, C.c_uint64, C.c_int, C.c_double,
                              C.POINTER(C.c_int8), _dp, _dp]
    L.or_subsweep.restype = C.c_int64
    L.or_serial_create.argtypes = [C.POINTER(OrSys)]
    L.or_serial_create.restype = C.c_void_p
    L.or_serial_destroy.argtypes = [C.c_void_p]
    L.or_serial_field.argtypes = [C.c_void_p, _dp, _dp]
    L.or_serial_sweep.argtypes = [C.c_void_p, C.POINTER(OrSys), C.POINTER(OrClass), _dp, _dp, C.c_uint64,
                                  C.c_double, C.c_int, _dp]
    L.or_serial_sweep.restype = C.c_int64
    L.or_init_state.argtypes = [C.POINTER(OrSys), C.POINTER(OrClass), C.c_int, _dp, _dp]
    L.or_run.argtypes = [C.POINTER(OrSys), C.POINTER(OrClass), C.c_void_p, _dp, C.c_uint64, C.c_int64,
                         C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int64), _dp]


def _ptr(a, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t))


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return [o[i] for i in range(4)]


def u01(x):
    return lib().or_u01(int(x) & 0xFFFFFFFF)


def meanfield(model, T, Tc, mu=MUB):
    me, ic = C.c_double(), C.c_double()
    lib().or_meanfield(int(model), float(T), float(Tc), float(mu), C.byref(me), C.byref(ic))
    return me.value, ic.value


def newell(X, Y, Z, hx, hy, hz, kind="auto", order=6):
    out = (C.c_double * 6)()
    if kind == "auto":
        lib().or_newell(X, Y, Z, hx, hy, hz, out)
    elif kind == "exact":
        lib().or_newell_exact(X, Y, Z, hx, hy, hz, out)
    else:
        lib().or_newell_far(X, Y, Z, hx, hy, hz, int(order), out)
    return np.array(out[:])


def dinvr(a, b, c, x, y, z):
    return lib().or_dinvr(a, b, c, x, y, z)


def demag_direct(grid, cell, m):
    nx, ny, nz = grid
    m = np.ascontiguousarray(m, dtype=np.float64).reshape(3, -1)
    h = np.zeros_like(m)
    lib().or_demag_direct(nx, ny, nz, *map(float, cell), _ptr(m), _ptr(h))
    return h


def demag_direct_at(grid, cell, m, cells):
    nx, ny, nz = grid
    m = np.ascontiguousarray(m, dtype=np.float64).reshape(3, -1)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((len(cells), 3))
    lib().or_demag_direct_at(nx, ny, nz, *map(float, cell), _ptr(m), _ptr(cells, C.c_int64), len(cells), _ptr(out))
    return out


class DemagPlan:
    def __init__(self, grid, cell):
        self.grid = tuple(grid)
        self._p = lib().or_demag_plan_create(*map(int, grid), *map(float, cell))

    def __call__(self, m):
        m = np.ascontiguousarray(m, dtype=np.float64).reshape(3, -1)
        h = np.zeros_like(m)
        lib().or_demag_plan_apply(self._p, _ptr(m), _ptr(h))
        return h

    def __del__(self):
        if getattr(self, "_p", None):
            lib().or_demag_plan_destroy(self._p)
            self._p = None


class System:
    """One chain: grid, cell, material (one class or per-grain classes), run settings.

    Mirrors the quantities the paper uses; every number is FP64.
    """

    def __init__(self, grid, cell, Ms0, A0, K1, Tc, T, D0=0.0, K2=0.0, easy_axis=(0, 0, 1), B=(0, 0, 0),
                 mf=1, mu=MUB, lenmode=0, demag=False, refresh_per_sweep=2, seed=0, chain_id=0,
                 sigma_fixed=0.0, cls=None, ea=None, K1s=None, K2s=None, Tcs=None, bscale=1.0, Tcl=None,
                 cubic_axes=None, kscale=False):
        self.grid = tuple(int(v) for v in grid)
        self.cell = tuple(float(v) for v in cell)
        self.N = int(np.prod(self.grid))
        if cls is None:
            self.nclass = 1
            self._ea = np.array(easy_axis, dtype=np.float64).reshape(1, 3)
            self._ea = self._ea / np.linalg.norm(self._ea)
            self._K1 = np.array([K1], dtype=np.float64)
            self._K2 = np.array([K2], dtype=np.float64)
            self._Tc = np.array([Tc], dtype=np.float64)
            self._cls = None
        else:
            self._cls = np.ascontiguousarray(cls, dtype=np.uint32)
            self.nclass = int(len(Tcs))
            self._ea = np.ascontiguousarray(ea, dtype=np.float64).reshape(-1, 3)
            self._K1 = np.ascontiguousarray(K1s, dtype=np.float64)
            self._K2 = np.ascontiguousarray(K2s if K2s is not None else np.zeros(self.nclass), dtype=np.float64)
            self._Tc = np.ascontiguousarray(Tcs, dtype=np.float64)
        s = OrSys()
        s.nx, s.ny, s.nz = self.grid
        s.hx, s.hy, s.hz = self.cell
        s.Ms0, s.A0, s.D0, s.T = float(Ms0), float(A0), float(D0), float(T)
        s.B[0], s.B[1], s.B[2] = [float(v) for v in B]
        s.mf, s.mu, s.lenmode = int(mf), float(mu), int(lenmode)
        s.demag, s.refresh_per_sweep = int(bool(demag)), int(refresh_per_sweep)
        s.seed, s.chain_id, s.sigma_fixed = int(seed), int(chain_id), float(sigma_fixed)
        s.nclass = self.nclass
        s.cls = _ptr(self._cls, C.c_uint32) if self._cls is not None else C.POINTER(C.c_uint32)()
        s.ea, s.K1, s.K2, s.Tc = _ptr(self._ea), _ptr(self._K1), _ptr(self._K2), _ptr(self._Tc)
        s.bscale = float(bscale)
        # per-class temperatures (non-uniform temperature profile), or None: all at T
        self._Tcl = None if Tcl is None else np.ascontiguousarray(Tcl, dtype=np.float64)
        if self._Tcl is not None:
            assert self._Tcl.shape == (self.nclass,)
        s.Tcl = _ptr(self._Tcl) if self._Tcl is not None else C.POINTER(C.c_double)()
        # cubic anisotropy (Eq. 12): (nclass, 3, 3) orthonormal crystal axes as rows (or (3, 3) for
        # all classes); K1/K2 (K1s/K2s) are then the cubic constants.  kscale: me^{l(l+1)/2} law.
        self._cax = None
        if cubic_axes is not None:
            ax = np.asarray(cubic_axes, dtype=np.float64)
            if ax.shape == (3, 3):
                ax = np.broadcast_to(ax, (self.nclass, 3, 3))
            assert ax.shape == (self.nclass, 3, 3)
            assert np.allclose(np.einsum("kij,klj->kil", ax, ax), np.eye(3), atol=1e-12)
            self._cax = np.ascontiguousarray(ax)
        s.anis = 0 if self._cax is None else 1
        s.cax = _ptr(self._cax) if self._cax is not None else C.POINTER(C.c_double)()
        s.kscale = int(bool(kscale))
        self.s = s
        self.refresh()
        self._plan = None

    # -- setup --------------------------------------------------------
    def refresh(self):
        self.cc = (OrClass * self.nclass)()
        lib().or_class_coeffs(C.byref(self.s), self.cc)

    def set_field(self, B):
        self.s.B[0], self.s.B[1], self.s.B[2] = [float(v) for v in B]

    def set_temperature(self, T):
        self.s.T = float(T)
        self.refresh()

    def coeffs(self, c=0):
        o = self.cc[c]
        return {k: getattr(o, k) for k, _ in OrClass._fields_}

    @property
    def plan(self):
        if self._plan is None:
            self._plan = DemagPlan(self.grid, self.cell)
        return self._plan

    # -- state --------------------------------------------------------
    def init_state(self, kind="uniform", direction=(0, 0, 1)):
        m = np.zeros((3, self.N))
        d = (C.c_double * 3)(*[float(v) for v in direction])
        lib().or_init_state(C.byref(self.s), self.cc, 0 if kind == "uniform" else 1, d, _ptr(m))
        return m

    def demag(self, m, method="fft"):
        if method == "fft":
            return self.plan(m)
        return demag_direct(self.grid, self.cell, m)

    def delta_F(self, m, p, mB, h=None):
        m = np.ascontiguousarray(m, dtype=np.float64)
        out = np.zeros(6)
        hb = np.ascontiguousarray(h, dtype=np.float64) if h is not None else None
        mb = np.ascontiguousarray(mB, dtype=np.float64)
        lib().or_delta_F(C.byref(self.s), self.cc, _ptr(m), _ptr(hb) if hb is not None else None,
                         int(p), _ptr(mb), _ptr(out))
        return out

    def energy(self, m, h=None, fresh_demag=True):
        m = np.ascontiguousarray(m, dtype=np.float64)
        if h is None and fresh_demag and self.s.demag:
            h = self.demag(m)
        out = np.zeros(6)
        hb = np.ascontiguousarray(h, dtype=np.float64) if h is not None else None
        lib().or_energy(C.byref(self.s), self.cc, _ptr(m), _ptr(hb) if hb is not None else None, _ptr(out))
        return out

    def subsweep(self, m, sweep, colour, cone_deg, h=None):
        """One colour pass in place on a copy; returns (m_new, acc, margin, mB)."""
        m = np.array(m, dtype=np.float64, order="C").reshape(3, -1)
        acc = np.zeros(self.N, dtype=np.int8)
        margin = np.zeros(self.N)
        mB = np.zeros((3, self.N))
        hb = np.ascontiguousarray(h, dtype=np.float64) if h is not None else None
        n = lib().or_subsweep(C.byref(self.s), self.cc, _ptr(m), _ptr(hb) if hb is not None else None,
                              int(sweep), int(colour), float(cone_deg), _ptr(acc, C.c_int8), _ptr(margin), _ptr(mB))
        return m, acc, margin, mB, int(n)

    def serial_field(self, m):
        """h = -N*m by the direct sum over the serial run's tensor table."""
        m = np.ascontiguousarray(m, dtype=np.float64).reshape(3, -1)
        h = np.zeros_like(m)
        lib().or_serial_field(self._serial_table(), _ptr(m), _ptr(h))
        return h

    def __del__(self):
        if getattr(self, "_ser", None) is not None:
            lib().or_serial_destroy(self._ser)
            self._ser = None

    def _serial_table(self):
        if getattr(self, "_ser", None) is None:
            self._ser = lib().or_serial_create(C.byref(self.s))
        return self._ser

    def serial_run(self, m, n, sweep0=0, cone_deg=30, adapt_every=0, window=0, h=None, self_term=False):
        """n serial sweeps with the demag field kept current, in place on m (and
        on h, the current field, computed fresh when None); self_term: exact
        total-energy change (adds the cell's self term to Eq. 14).  Returns
        (series[n,5], cone_deg, window, h, accepted dF in J).  The cone rule is
        that of run()."""
        assert m.dtype == np.float64 and m.flags.c_contiguous
        q = self._serial_table()
        if h is None:
            h = self.serial_field(m) if self.s.demag else np.zeros_like(m)
        assert h.dtype == np.float64 and h.flags.c_contiguous
        series = np.zeros((int(n), 5))
        dE = C.c_double(0.0)
        cd, win = int(cone_deg), int(window)
        for i in range(int(n)):
            sw = int(sweep0) + i
            nacc = lib().or_serial_sweep(q, C.byref(self.s), self.cc, _ptr(m), _ptr(h), sw, float(cd), int(bool(self_term)),
                                         C.byref(dE))
            win += nacc
            series[i, :3] = m.mean(axis=1)
            series[i, 3] = (m * m).sum(axis=0).mean()
            series[i, 4] = nacc
            if adapt_every > 0 and (sw + 1) % adapt_every == 0:
                tot = adapt_every * self.N
                if 100 * win > 55 * tot and cd < 180:
                    cd += 1
                elif 100 * win < 45 * tot and cd > 1:
                    cd -= 1
                win = 0
        return series, cd, win, h, dE.value

    def run(self, m, n, sweep0=0, cone_deg=30, adapt_every=0, window=0):
        """n full sweeps in place; returns (series[n,5], cone_deg, window)."""
        assert m.dtype == np.float64 and m.flags.c_contiguous
        cd = C.c_int32(int(cone_deg))
        win = C.c_int64(int(window))
        series = np.zeros((int(n), 5))
        plan = self.plan._p if self.s.demag else None
        lib().or_run(C.byref(self.s), self.cc, plan, _ptr(m), int(sweep0), int(n), C.byref(cd),
                     int(adapt_every), C.byref(win), _ptr(series))
        return series, cd.value, win.value
