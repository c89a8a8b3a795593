"""CPU oracle for the SU(2) Wilson-action heat-bath sweep (test infrastructure).

Only the tests, the package's smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product path (the HIP library and its
Python binding) never does, and the two share no code: the lattice chain is
plain C in ``su2_oracle.c`` (FP64 arithmetic, FP32 link storage as the paper
fixes in Sec. 2.4), wrapped here with ctypes; the learned-proposal pieces are
plain NumPy in ``cdf.py`` and ``mlp.py``.

Link arrays on this side are float64 numpy arrays of shape [V, 4, 4] indexed
(site lex, direction mu, quaternion component), lex = x0 + L0*(x1 + L1*(x2 +
L2*x3)), direction 3 = time.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libsu2_oracle.so")
_lib = None

COLD, HOT = 0, 1


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIBPATH)
    i32p = ctypes.POINTER(ctypes.c_int32)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    dp = ctypes.POINTER(ctypes.c_double)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    i8p = ctypes.POINTER(ctypes.c_int8)
    lib.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_uniform.argtypes = [ctypes.c_uint32]
    lib.oracle_uniform.restype = ctypes.c_double
    lib.oracle_qmul.argtypes = [dp, dp, dp]
    lib.oracle_qmul.restype = None
    lib.oracle_staple.argtypes = [i32p, dp, ctypes.c_long, ctypes.c_int, dp]
    lib.oracle_staple.restype = None
    lib.oracle_kp_draw.argtypes = [ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                   ctypes.c_int, ctypes.c_uint32, ctypes.c_int, dp, dp, dp]
    lib.oracle_kp_draw.restype = ctypes.c_int
    lib.oracle_creutz_draw.argtypes = lib.oracle_kp_draw.argtypes
    lib.oracle_creutz_draw.restype = ctypes.c_int
    lib.oracle_init.argtypes = [i32p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, dp]
    lib.oracle_init.restype = ctypes.c_int
    lib.oracle_init_sites.argtypes = [i32p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int64), ctypes.c_long, dp]
    lib.oracle_init_sites.restype = ctypes.c_int
    lib.oracle_pass.argtypes = [i32p, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, i8p,
                                dp, dp, u64p]
    lib.oracle_pass.restype = ctypes.c_int
    lib.oracle_update_sites.argtypes = [i32p, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_double, dp,
                                        ctypes.POINTER(ctypes.c_int64), ctypes.c_long, dp, i8p, dp]
    lib.oracle_update_sites.restype = ctypes.c_int
    lib.oracle_sweep.argtypes = [i32p, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                 ctypes.c_int, ctypes.c_double, dp, u64p]
    lib.oracle_sweep.restype = ctypes.c_int
    lib.oracle_plaquette.argtypes = [i32p, dp, dp]
    lib.oracle_plaquette.restype = ctypes.c_int
    lib.oracle_polyakov.argtypes = [i32p, dp, dp]
    lib.oracle_polyakov.restype = ctypes.c_int
    lib.oracle_staple_action.argtypes = [i32p, dp, dp]
    lib.oracle_staple_action.restype = ctypes.c_int
    lib.oracle_pass_imh.argtypes = [i32p, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int,
                                    ctypes.c_double, i8p, dp, u64p]
    lib.oracle_pass_imh.restype = ctypes.c_int
    lib.oracle_sweep_imh.argtypes = [i32p, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                     ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_double, u64p]
    lib.oracle_sweep_imh.restype = ctypes.c_int
    lib.oracle_polyakov_field.argtypes = [i32p, dp, dp]
    lib.oracle_polyakov_field.restype = ctypes.c_int
    lib.oracle_or_pass.argtypes = [i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
    lib.oracle_or_pass.restype = ctypes.c_int
    lib.oracle_or_sweep.argtypes = [i32p, ctypes.c_int, dp]
    lib.oracle_or_sweep.restype = ctypes.c_int
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _dims(dims):
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
    if d.shape != (4,):
        raise ValueError("dims must have 4 entries")
    return d


def volume(dims):
    return int(np.prod(np.asarray(dims, dtype=np.int64)))


def philox4x32_10(counter, key):
    """Philox-4x32-10 block for counter (4 x u32) and key (2 x u32)."""
    lib = _load()
    c = np.ascontiguousarray(np.asarray(counter, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    o = np.zeros(4, dtype=np.uint32)
    lib.oracle_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                             _ptr(o, ctypes.c_uint32))
    return o


def num_threads():
    return int(_load().oracle_num_threads())


def uniform(word):
    return _load().oracle_uniform(int(word))


def qmul(a, b):
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    c = np.zeros(4)
    lib.oracle_qmul(_ptr(a, ctypes.c_double), _ptr(b, ctypes.c_double), _ptr(c, ctypes.c_double))
    return c


def init(dims, seed, start, prec32=True):
    """Cold (start=0) or hot (start=1) lattice, float64 [V, 4, 4]."""
    lib = _load()
    d = _dims(dims)
    U = np.zeros((volume(dims), 4, 4))
    rc = lib.oracle_init(_ptr(d, ctypes.c_int32), ctypes.c_uint64(seed), int(start),
                         int(bool(prec32)), _ptr(U, ctypes.c_double))
    if rc:
        raise ValueError("oracle_init rejected its arguments")
    return U


def init_sites(dims, seed, start, sites, prec32=True):
    """The links init() gives the listed sites, float64 [n, 4, 4], without
    forming the lattice (for lattices too large to hold)."""
    lib = _load()
    d = _dims(dims)
    sites = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    out = np.zeros((len(sites), 4, 4))
    rc = lib.oracle_init_sites(_ptr(d, ctypes.c_int32), ctypes.c_uint64(seed), int(start),
                               int(bool(prec32)), _ptr(sites, ctypes.c_int64), len(sites),
                               _ptr(out, ctypes.c_double))
    if rc:
        raise ValueError("oracle_init_sites rejected its arguments")
    return out


def _links(U):
    U = np.ascontiguousarray(U, dtype=np.float64)
    if U.ndim != 3 or U.shape[1:] != (4, 4):
        raise ValueError("links must have shape [V, 4, 4]")
    return U


def staple(dims, U, lex, mu):
    lib = _load()
    d = _dims(dims)
    U = _links(U)
    w = np.zeros(4)
    lib.oracle_staple(_ptr(d, ctypes.c_int32), _ptr(U, ctypes.c_double), int(lex), int(mu),
                      _ptr(w, ctypes.c_double))
    return w


def _draw(fn, alpha, seed, site, mu, sweep, prec32):
    a0 = ctypes.c_double(np.nan)
    am = ctypes.c_double(np.nan)
    m = ctypes.c_double(np.nan)
    t = fn(float(alpha), ctypes.c_uint64(seed), int(site), int(mu), int(sweep),
           int(bool(prec32)), ctypes.byref(a0), ctypes.byref(am), ctypes.byref(m))
    return t, a0.value, am.value, m.value


def kp_draw(alpha, seed, site, mu, sweep, prec32=True):
    """One capped KP draw.  Returns (attempt index or -1, x0, |a|, margin)."""
    return _draw(_load().oracle_kp_draw, alpha, seed, site, mu, sweep, prec32)


def creutz_draw(alpha, seed, site, mu, sweep, prec32=True):
    """One capped Creutz draw (the heat-bath below the small-alpha switch).
    Returns (attempt index or -1, x0, |a|, margin)."""
    return _draw(_load().oracle_creutz_draw, alpha, seed, site, mu, sweep, prec32)


class PassResult:
    def __init__(self, tries, margin, attempts, failures, knorm=None, x0=None):
        self.tries = tries
        self.margin = margin
        self.attempts = attempts
        self.failures = failures
        self.knorm = knorm   # |w| of each updated link (diag=True), else None
        self.x0 = x0         # its accepted x0 (NaN: Haar branch or cap failure)


def heatbath_pass(dims, U, beta, seed, sweep, parity, mu, prec32=True, creutz_below=0.0,
                  diag=False):
    """In-place heat-bath pass over links U_mu(x), parity(x) == parity
    (Creutz's draw where alpha < creutz_below).  diag=True also returns, per
    updated site, the staple norm |w| and the accepted x0."""
    lib = _load()
    d = _dims(dims)
    if not (isinstance(U, np.ndarray) and U.dtype == np.float64 and U.flags.c_contiguous):
        raise ValueError("U must be a C-contiguous float64 array")
    V = volume(dims)
    tries = np.full(V, -1, dtype=np.int8)
    margin = np.full(V, np.nan)
    stats = np.zeros(2, dtype=np.uint64)
    dg = np.full((V, 2), np.nan) if diag else None
    rc = lib.oracle_pass(_ptr(d, ctypes.c_int32), float(beta), ctypes.c_uint64(seed), int(sweep),
                         int(parity), int(mu), int(bool(prec32)), float(creutz_below),
                         _ptr(U, ctypes.c_double), _ptr(tries, ctypes.c_int8), _ptr(margin, ctypes.c_double),
                         _ptr(dg, ctypes.c_double) if diag else None, _ptr(stats, ctypes.c_uint64))
    if rc:
        raise ValueError("oracle_pass rejected its arguments")
    return PassResult(tries, margin, int(stats[0]), int(stats[1]),
                      dg[:, 0] if diag else None, dg[:, 1] if diag else None)


def update_sites(dims, U, beta, seed, sweep_index, mu, sites, prec32=True, creutz_below=0.0):
    """New values of U_mu at the listed sites (one parity) as a pass at
    sweep_index would write them; U is not modified.  Returns (links [n,4],
    tries [n], margin [n])."""
    lib = _load()
    d = _dims(dims)
    U = _links(U)
    sites = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    n = len(sites)
    out = np.zeros((n, 4))
    tries = np.full(n, -1, dtype=np.int8)
    margin = np.full(n, np.nan)
    rc = lib.oracle_update_sites(_ptr(d, ctypes.c_int32), float(beta), ctypes.c_uint64(seed),
                                 int(sweep_index), int(mu), int(bool(prec32)), float(creutz_below),
                                 _ptr(U, ctypes.c_double), _ptr(sites, ctypes.c_int64), n,
                                 _ptr(out, ctypes.c_double), _ptr(tries, ctypes.c_int8),
                                 _ptr(margin, ctypes.c_double))
    if rc:
        raise ValueError("oracle_update_sites rejected its arguments")
    return out, tries, margin


def _table(table):
    t = np.ascontiguousarray(np.asarray(table, dtype=np.float64))
    if t.ndim != 2 or t.shape[1] != 33 or t.shape[0] < 2:
        raise ValueError("knot table must have shape [G >= 2, 33]")
    return t


def imh_pass(dims, U, beta, seed, sweep_index, parity, mu, table, alpha_max=40.0, prec32=True):
    """In-place pass with the learned independence-Metropolis proposal.
    Returns (result codes per site, margins, proposals, accepts); codes 10 =
    accepted, 11 = rejected (x0 kept, direction redrawn), 0..9 = plain
    heat-bath codes."""
    lib = _load()
    d = _dims(dims)
    if not (isinstance(U, np.ndarray) and U.dtype == np.float64 and U.flags.c_contiguous):
        raise ValueError("U must be a C-contiguous float64 array")
    t = _table(table)
    V = volume(dims)
    res = np.full(V, -1, dtype=np.int8)
    margin = np.full(V, np.nan)
    stats = np.zeros(2, dtype=np.uint64)
    rc = lib.oracle_pass_imh(_ptr(d, ctypes.c_int32), float(beta), ctypes.c_uint64(seed),
                             int(sweep_index), int(parity), int(mu), int(bool(prec32)),
                             _ptr(U, ctypes.c_double), _ptr(t, ctypes.c_double), len(t),
                             float(alpha_max), _ptr(res, ctypes.c_int8),
                             _ptr(margin, ctypes.c_double), _ptr(stats, ctypes.c_uint64))
    if rc:
        raise ValueError("oracle_pass_imh rejected its arguments")
    return res, margin, int(stats[0]), int(stats[1])


def imh_sweep(dims, U, beta, seed, sweep_index, table, alpha_max=40.0, prec32=True):
    lib = _load()
    d = _dims(dims)
    t = _table(table)
    stats = np.zeros(2, dtype=np.uint64)
    rc = lib.oracle_sweep_imh(_ptr(d, ctypes.c_int32), float(beta), ctypes.c_uint64(seed),
                              int(sweep_index), int(bool(prec32)), _ptr(U, ctypes.c_double),
                              _ptr(t, ctypes.c_double), len(t), float(alpha_max),
                              _ptr(stats, ctypes.c_uint64))
    if rc:
        raise ValueError("oracle_sweep_imh rejected its arguments")
    return int(stats[0]), int(stats[1])


def sweep(dims, U, beta, seed, sweep_index, prec32=True, creutz_below=0.0):
    """In-place full sweep; returns (attempts, cap failures)."""
    lib = _load()
    d = _dims(dims)
    if not (isinstance(U, np.ndarray) and U.dtype == np.float64 and U.flags.c_contiguous):
        raise ValueError("U must be a C-contiguous float64 array")
    stats = np.zeros(2, dtype=np.uint64)
    rc = lib.oracle_sweep(_ptr(d, ctypes.c_int32), float(beta), ctypes.c_uint64(seed),
                          int(sweep_index), int(bool(prec32)), float(creutz_below),
                          _ptr(U, ctypes.c_double), _ptr(stats, ctypes.c_uint64))
    if rc:
        raise ValueError("oracle_sweep rejected its arguments")
    return int(stats[0]), int(stats[1])


def or_pass(dims, U, parity, mu, prec32=True, diag=False):
    """In-place overrelaxation pass: U_mu(x) -> V U^dag V, V = w/|w|, on the
    sites of one parity (links with w = 0 kept).  diag=True returns the staple
    norm |w| per site (NaN off the pass's parity)."""
    lib = _load()
    d = _dims(dims)
    if not (isinstance(U, np.ndarray) and U.dtype == np.float64 and U.flags.c_contiguous):
        raise ValueError("U must be a C-contiguous float64 array")
    kn = np.full(volume(dims), np.nan) if diag else None
    if lib.oracle_or_pass(_ptr(d, ctypes.c_int32), int(parity), int(mu), int(bool(prec32)),
                          _ptr(U, ctypes.c_double), _ptr(kn, ctypes.c_double) if diag else None):
        raise ValueError("oracle_or_pass rejected its arguments")
    return kn


def or_sweep(dims, U, prec32=True):
    """In-place overrelaxation sweep (odd sites for mu = 0..3, then even)."""
    lib = _load()
    d = _dims(dims)
    if not (isinstance(U, np.ndarray) and U.dtype == np.float64 and U.flags.c_contiguous):
        raise ValueError("U must be a C-contiguous float64 array")
    if lib.oracle_or_sweep(_ptr(d, ctypes.c_int32), int(bool(prec32)), _ptr(U, ctypes.c_double)):
        raise ValueError("oracle_or_sweep rejected its arguments")


def plaquette(dims, U):
    """(P, P_spatial, P_temporal) in FP64."""
    lib = _load()
    d = _dims(dims)
    U = _links(U)
    out = np.zeros(3)
    if lib.oracle_plaquette(_ptr(d, ctypes.c_int32), _ptr(U, ctypes.c_double),
                            _ptr(out, ctypes.c_double)):
        raise ValueError("bad dims")
    return out


def polyakov(dims, U):
    lib = _load()
    d = _dims(dims)
    U = _links(U)
    out = ctypes.c_double(np.nan)
    if lib.oracle_polyakov(_ptr(d, ctypes.c_int32), _ptr(U, ctypes.c_double), ctypes.byref(out)):
        raise ValueError("bad dims")
    return out.value


def polyakov_field(dims, U):
    """(1/2)Tr of the ordered product of U_3 over t at every spatial site
    (lex x0 + L0 (x1 + L1 x2)), FP64."""
    lib = _load()
    d = _dims(dims)
    U = _links(U)
    out = np.empty(int(d[0]) * int(d[1]) * int(d[2]))
    if lib.oracle_polyakov_field(_ptr(d, ctypes.c_int32), _ptr(U, ctypes.c_double), _ptr(out, ctypes.c_double)):
        raise ValueError("bad dims")
    return out


def polyakov_correlator(dims, U, rmax):
    """C(r) = mean over spatial sites xs and the three spatial directions i of
    L(xs) L(xs + r e_i), r = 0 .. rmax (periodic), from polyakov_field."""
    L0, L1, L2 = (int(v) for v in dims[:3])
    F = polyakov_field(dims, U).reshape(L2, L1, L0)
    out = np.empty(rmax + 1)
    for r in range(rmax + 1):
        out[r] = np.mean(F * (np.roll(F, -r, axis=2) + np.roll(F, -r, axis=1) + np.roll(F, -r, axis=0))) / 3.0
    return out


def staple_action(dims, U):
    lib = _load()
    d = _dims(dims)
    U = _links(U)
    out = ctypes.c_double(np.nan)
    if lib.oracle_staple_action(_ptr(d, ctypes.c_int32), _ptr(U, ctypes.c_double),
                                ctypes.byref(out)):
        raise ValueError("bad dims")
    return out.value


class Chain:
    """A running oracle chain: links + sweep counter, mirroring the library's
    global context (init, sweep(n), plaquette, polyakov, links)."""

    def __init__(self, dims, beta, seed, start, prec32=True, creutz_below=0.0):
        self.dims = tuple(int(x) for x in dims)
        self.beta = float(beta)
        self.seed = int(seed)
        self.prec32 = bool(prec32)
        self.creutz_below = float(creutz_below)
        self.U = init(dims, seed, start, prec32)
        self.s = 0
        self.attempts = 0
        self.failures = 0

    def sweep(self, n=1):
        for _ in range(n):
            a, f = sweep(self.dims, self.U, self.beta, self.seed, self.s, self.prec32, self.creutz_below)
            self.attempts += a
            self.failures += f
            self.s += 1

    def plaquette(self):
        return plaquette(self.dims, self.U)

    def polyakov(self):
        return polyakov(self.dims, self.U)
