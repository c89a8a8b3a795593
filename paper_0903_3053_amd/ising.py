"""Thin ctypes binding of the 2-D Ising entry points of libsu2.so
(include/ising.h): the same names, argument marshalling only; every step runs
in the library's HIP kernels.  Spins are int8 (+1 / -1) in lex order x + L0 y."""
import ctypes

import numpy as np

from . import su2

# every symbol include/ising.h declares
EXPORTS = ("ising_init", "ising_init_ex", "ising_layout", "ising_sweep", "ising_observables", "ising_spins",
           "ising_set_spins", "ising_sweep_index", "ising_accepted", "ising_last_error", "ising_finalize")
COLD, HOT = 0, 1
LAYOUT_AUTO, LAYOUT_BYTES, LAYOUT_BITS = 0, 1, 2

_ready = False


def load():
    global _ready
    lib = su2.load()
    if not _ready:
        i32p = ctypes.POINTER(ctypes.c_int32)
        i8p = ctypes.POINTER(ctypes.c_int8)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        dp = ctypes.POINTER(ctypes.c_double)
        sig = {
            "ising_init": ([i32p, ctypes.c_double, ctypes.c_uint64, ctypes.c_int32], ctypes.c_int),
            "ising_init_ex": ([i32p, ctypes.c_double, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32],
                              ctypes.c_int),
            "ising_layout": ([i32p], ctypes.c_int),
            "ising_sweep": ([ctypes.c_int32], ctypes.c_int),
            "ising_observables": ([dp], ctypes.c_int),
            "ising_spins": ([i8p, ctypes.c_size_t], ctypes.c_int),
            "ising_set_spins": ([i8p, ctypes.c_size_t, ctypes.c_uint64], ctypes.c_int),
            "ising_sweep_index": ([u64p], ctypes.c_int),
            "ising_accepted": ([u64p], ctypes.c_int),
            "ising_last_error": ([], ctypes.c_char_p),
            "ising_finalize": ([], None),
        }
        for name, (args, res) in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _ready = True
    return lib


class IsingError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ising error {code}: {msg}")
        self.code = code


_shape = {}


def _check(rc):
    if rc != su2.SU2_OK:
        raise IsingError(rc, load().ising_last_error().decode())


def ising_init(dims, beta, seed, start, layout=None):
    """layout None calls ising_init (auto); 0/1/2 call ising_init_ex."""
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
    if d.shape != (2,):
        raise ValueError("dims must have 2 entries")
    dp = d.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    if layout is None:
        _check(load().ising_init(dp, float(beta), ctypes.c_uint64(seed), int(start)))
    else:
        _check(load().ising_init_ex(dp, float(beta), ctypes.c_uint64(seed), int(start), int(layout)))
    _shape["n"] = int(d[0]) * int(d[1])


def ising_init_ex(dims, beta, seed, start, layout):
    ising_init(dims, beta, seed, start, layout)


def ising_layout():
    out = ctypes.c_int32(0)
    _check(load().ising_layout(ctypes.byref(out)))
    return out.value


def ising_sweep(n=1):
    _check(load().ising_sweep(int(n)))


def ising_observables():
    """(energy per site, magnetisation per site)."""
    out = np.zeros(2)
    _check(load().ising_observables(out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return float(out[0]), float(out[1])


def ising_spins():
    out = np.empty(_shape.get("n", 0), dtype=np.int8)
    _check(load().ising_spins(out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), out.size))
    return out


def ising_set_spins(spins, sweep_index):
    s = np.ascontiguousarray(spins, dtype=np.int8)
    _check(load().ising_set_spins(s.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), s.size,
                                  ctypes.c_uint64(sweep_index)))


def ising_sweep_index():
    out = ctypes.c_uint64(0)
    _check(load().ising_sweep_index(ctypes.byref(out)))
    return out.value


def ising_accepted():
    out = ctypes.c_uint64(0)
    _check(load().ising_accepted(ctypes.byref(out)))
    return out.value


def ising_finalize():
    load().ising_finalize()
