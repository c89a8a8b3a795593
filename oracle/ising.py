"""Python face of the 2-D Ising oracle (ising_oracle.c): Metropolis on a
red-black partition of an L0 x L1 periodic lattice, H = -sum_<ij> s_i s_j
(Sec. 2.3, Eq. (1)).  Test infrastructure only, like the rest of oracle/.
Spins are int8 (+1 / -1) in lex order x + L0 y."""
import ctypes

import numpy as np

from . import _load as _load_lib

_ready = False


def _lib():
    global _ready
    lib = _load_lib()
    if not _ready:
        i32p = ctypes.POINTER(ctypes.c_int32)
        i8p = ctypes.POINTER(ctypes.c_int8)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_ising_init.argtypes = [i32p, ctypes.c_uint64, ctypes.c_int, i8p]
        lib.oracle_ising_init.restype = ctypes.c_int
        lib.oracle_ising_sweep.argtypes = [i32p, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                           ctypes.c_int, i8p, ctypes.POINTER(ctypes.c_uint64)]
        lib.oracle_ising_sweep.restype = ctypes.c_int
        lib.oracle_ising_observables.argtypes = [i32p, i8p, dp]
        lib.oracle_ising_observables.restype = ctypes.c_int
        _ready = True
    return lib


def _dims(dims):
    return np.ascontiguousarray(dims, dtype=np.int32)


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def init(dims, seed, start):
    """start 0 = cold (all +1), 1 = hot (Philox)."""
    d = _dims(dims)
    s = np.empty(int(d[0]) * int(d[1]), dtype=np.int8)
    if _lib().oracle_ising_init(_p(d, ctypes.c_int32), ctypes.c_uint64(seed), int(start), _p(s, ctypes.c_int8)):
        raise ValueError("oracle_ising_init rejected its arguments")
    return s


def sweep(dims, s, beta, seed, sweep0, n=1):
    """n Metropolis sweeps in place from sweep index sweep0; returns the
    number of accepted flips."""
    d = _dims(dims)
    if not (isinstance(s, np.ndarray) and s.dtype == np.int8 and s.flags.c_contiguous):
        raise ValueError("spins must be a C-contiguous int8 array")
    acc = ctypes.c_uint64(0)
    if _lib().oracle_ising_sweep(_p(d, ctypes.c_int32), float(beta), ctypes.c_uint64(seed), int(sweep0),
                                 int(n), _p(s, ctypes.c_int8), ctypes.byref(acc)):
        raise ValueError("oracle_ising_sweep rejected its arguments")
    return int(acc.value)


def observables(dims, s):
    """(energy per site, magnetisation per site), exact integer sums."""
    d = _dims(dims)
    out = np.zeros(2)
    if _lib().oracle_ising_observables(_p(d, ctypes.c_int32), _p(s, ctypes.c_int8), _p(out, ctypes.c_double)):
        raise ValueError("oracle_ising_observables rejected its arguments")
    return float(out[0]), float(out[1])
