"""Thin ctypes binding of libsu2.so (include/su2.h): the same entry points,
argument marshalling only.  Every step of the path runs in the library's HIP
kernels; there is no fallback, and a missing library raises.

PyTorch supplies device memory and streams: by default the link field is a
torch CUDA tensor handed to su2_init_ex, and set_stream() accepts a
torch.cuda.Stream.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libsu2.so")

SU2_OK, SU2_EINVAL, SU2_ESTATE, SU2_ENOMEM, SU2_EDEVICE = 0, -1, -2, -3, -4
COLD, HOT = 0, 1
FUSED_PAIRS = 300  # su2_set_plan order kind: each parity as two fused launches
# su2_set_creutz switch at which Kennedy-Pendleton and Creutz attempts are
# accepted equally often (71%): sqrt(2 pi a) e^-a I1(a) = pi I1(a) / (2 sinh a)
CREUTZ_SWITCH = 1.6847376

# every symbol include/su2.h declares
EXPORTS = (
    "su2_init", "su2_init_ex", "su2_bind", "su2_sweep", "su2_sweep_measured", "su2_pass", "su2_overrelax",
    "su2_overrelax_pass", "su2_plaquette", "su2_plaquette_st", "su2_polyakov", "su2_polyakov_correlator",
    "su2_polyakov_correlator_noalloc", "su2_measure_device", "su2_sweep_measure", "su2_links", "su2_set_links",
    "su2_sweep_index", "su2_counters", "su2_set_stream", "su2_set_plan", "su2_tune", "su2_philox",
    "su2_synchronize", "su2_last_error",
    "su2_finalize", "su2_batch_init", "su2_batch_sweep", "su2_batch_set_mode", "su2_batch_tune",
    "su2_batch_set_spin_limit", "su2_batch_plaquette", "su2_batch_links", "su2_batch_counters",
    "su2_batch_sweep_index", "su2_batch_last_error", "su2_batch_finalize",
    "su2_cdf_knots", "su2_mlp_set_params", "su2_mlp_get_params", "su2_mlp_forward",
    "su2_mlp_loss_grad", "su2_mlp_train", "su2_mlp_tabulate", "su2_mlp_table", "su2_cdf_tabulate",
    "su2_mlp_last_error", "su2_set_proposal", "su2_set_creutz", "su2_set_wide_offsets", "su2_imh_counters",
)


class Su2Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"su2 error {code}: {msg}")
        self.code = code


_lib = None
_keep = {}  # torch objects the library points into


def load():
    """Load libsu2.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise ImportError(f"{LIBPATH} is missing: build it with paper_0903_3053_amd/build.py")
    # PyTorch ships its own HIP runtime under the same soname (libamdhip64.so.7).
    # Importing torch first makes libsu2.so bind to that already-loaded copy, so
    # the process holds one HIP runtime and torch memory/streams are valid here.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIBPATH)
    i32p = ctypes.POINTER(ctypes.c_int32)
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    sig = {
        "su2_init": ([i32p, ctypes.c_double, ctypes.c_uint64, ctypes.c_int32], ctypes.c_int),
        "su2_init_ex": ([i32p, ctypes.c_double, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p,
                         ctypes.c_size_t], ctypes.c_int),
        "su2_bind": ([ctypes.c_void_p, ctypes.c_size_t], ctypes.c_int),
        "su2_sweep": ([ctypes.c_int32], ctypes.c_int),
        "su2_sweep_measured": ([ctypes.c_int32], ctypes.c_int),
        "su2_pass": ([ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
        "su2_overrelax": ([ctypes.c_int32], ctypes.c_int),
        "su2_polyakov_correlator": ([ctypes.c_int32, dp], ctypes.c_int),
        "su2_polyakov_correlator_noalloc": ([ctypes.c_int32, ctypes.c_void_p], ctypes.c_int),
        "su2_overrelax_pass": ([ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
        "su2_plaquette": ([], ctypes.c_double),
        "su2_plaquette_st": ([dp], ctypes.c_int),
        "su2_polyakov": ([dp], ctypes.c_int),
        "su2_measure_device": ([ctypes.c_void_p], ctypes.c_int),
        "su2_sweep_measure": ([ctypes.c_int32, ctypes.c_int32, dp], ctypes.c_int),
        "su2_links": ([fp, ctypes.c_size_t], ctypes.c_int),
        "su2_set_links": ([fp, ctypes.c_size_t, ctypes.c_uint64], ctypes.c_int),
        "su2_sweep_index": ([u64p], ctypes.c_int),
        "su2_counters": ([u64p], ctypes.c_int),
        "su2_set_stream": ([ctypes.c_void_p], ctypes.c_int),
        "su2_set_plan": ([ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
        "su2_tune": ([ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
        "su2_philox": ([ctypes.c_uint64, u32p, ctypes.c_size_t, u32p], ctypes.c_int),
        "su2_synchronize": ([], ctypes.c_int),
        "su2_last_error": ([], ctypes.c_char_p),
        "su2_finalize": ([], None),
        "su2_batch_init": ([ctypes.c_int32, i32p, dp, u64p, ctypes.c_int32], ctypes.c_int),
        "su2_batch_sweep": ([ctypes.c_int32], ctypes.c_int),
        "su2_batch_set_mode": ([ctypes.c_int32, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
        "su2_batch_tune": ([ctypes.c_int32, i32p], ctypes.c_int),
        "su2_batch_set_spin_limit": ([ctypes.c_uint64], ctypes.c_int),
        "su2_batch_plaquette": ([dp], ctypes.c_int),
        "su2_batch_links": ([ctypes.c_int32, fp, ctypes.c_size_t], ctypes.c_int),
        "su2_batch_counters": ([ctypes.c_int32, u64p], ctypes.c_int),
        "su2_batch_sweep_index": ([u64p], ctypes.c_int),
        "su2_batch_last_error": ([], ctypes.c_char_p),
        "su2_batch_finalize": ([], None),
        "su2_cdf_knots": ([dp, ctypes.c_int32, dp], ctypes.c_int),
        "su2_mlp_set_params": ([fp, ctypes.c_size_t], ctypes.c_int),
        "su2_mlp_get_params": ([fp, ctypes.POINTER(ctypes.c_uint16), ctypes.c_size_t], ctypes.c_int),
        "su2_mlp_forward": ([fp, ctypes.c_int32, fp], ctypes.c_int),
        "su2_mlp_loss_grad": ([fp, fp, ctypes.c_int32, fp, fp], ctypes.c_int),
        "su2_mlp_train": ([dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_float, fp],
                          ctypes.c_int),
        "su2_mlp_tabulate": ([ctypes.c_int32], ctypes.c_int),
        "su2_mlp_table": ([fp, ctypes.c_size_t], ctypes.c_int),
        "su2_cdf_tabulate": ([ctypes.c_int32], ctypes.c_int),
        "su2_mlp_last_error": ([], ctypes.c_char_p),
        "su2_set_proposal": ([ctypes.c_int32, ctypes.POINTER(ctypes.c_uint16), ctypes.c_size_t],
                             ctypes.c_int),
        "su2_set_creutz": ([ctypes.c_double], ctypes.c_int),
        "su2_set_wide_offsets": ([ctypes.c_int32], ctypes.c_int),
        "su2_imh_counters": ([u64p], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc):
    if rc != SU2_OK:
        raise Su2Error(rc, _lib.su2_last_error().decode())
    return rc


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _dims(dims):
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
    if d.shape != (4,):
        raise ValueError("dims must have 4 entries")
    return d


def su2_init(dims, beta, seed, start, torch_memory=True):
    """Create the lattice.  With torch_memory the link field is a torch CUDA
    tensor of 16*V float32 (kept alive here); otherwise the library allocates."""
    lib = load()
    d = _dims(dims)
    V = int(np.prod(d.astype(np.int64)))
    if torch_memory:
        import torch
        buf = torch.empty(16 * V, dtype=torch.float32, device="cuda")
        _keep["links"] = buf
        _check(lib.su2_init_ex(_ptr(d, ctypes.c_int32), float(beta), ctypes.c_uint64(seed),
                               int(start), ctypes.c_void_p(buf.data_ptr()), buf.numel() * 4))
    else:
        _keep.pop("links", None)
        _check(lib.su2_init(_ptr(d, ctypes.c_int32), float(beta), ctypes.c_uint64(seed),
                            int(start)))
    _keep["dims"] = tuple(int(x) for x in d)


def su2_init_ex(dims, beta, seed, start, dev_ptr, nbytes):
    lib = load()
    d = _dims(dims)
    _check(lib.su2_init_ex(_ptr(d, ctypes.c_int32), float(beta), ctypes.c_uint64(seed),
                           int(start), ctypes.c_void_p(dev_ptr), int(nbytes)))
    _keep["dims"] = tuple(int(x) for x in d)


def su2_bind(buf):
    """Move the links into a caller-owned device buffer: a torch CUDA tensor
    (kept alive here until the next init or finalize) of at least 64 V bytes."""
    _check(load().su2_bind(ctypes.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size()))
    _keep["links"] = buf


def su2_sweep(n=1):
    _check(load().su2_sweep(int(n)))


def su2_sweep_measured(n=1):
    _check(load().su2_sweep_measured(int(n)))


def su2_pass(parity, mu):
    _check(load().su2_pass(int(parity), int(mu)))


def su2_polyakov_correlator(rmax):
    """C(r), r = 0..rmax: <L(x) L(x + r e_i)> over spatial sites and directions."""
    out = np.zeros(int(rmax) + 1)
    _check(load().su2_polyakov_correlator(int(rmax), _ptr(out, ctypes.c_double)))
    return out


def su2_polyakov_correlator_noalloc(rmax, dev_out):
    """Enqueue C(0..rmax) into device memory without allocating: dev_out is a
    torch float64 CUDA tensor (its first rmax + 1 elements) or a raw address."""
    ptr = dev_out.data_ptr() if hasattr(dev_out, "data_ptr") else int(dev_out)
    _check(load().su2_polyakov_correlator_noalloc(int(rmax), ctypes.c_void_p(ptr)))


def su2_overrelax(n):
    """n overrelaxation sweeps (U -> V U^dag V about the staple direction)."""
    _check(load().su2_overrelax(int(n)))


def su2_overrelax_pass(parity, mu):
    _check(load().su2_overrelax_pass(int(parity), int(mu)))


def su2_plaquette():
    v = load().su2_plaquette()
    if np.isnan(v):
        raise Su2Error(-1, _lib.su2_last_error().decode())
    return v


def su2_plaquette_st():
    out = np.zeros(3)
    _check(load().su2_plaquette_st(_ptr(out, ctypes.c_double)))
    return out


def su2_polyakov():
    out = ctypes.c_double(np.nan)
    _check(load().su2_polyakov(ctypes.byref(out)))
    return out.value


def su2_measure_device(dev_out):
    """Enqueue (P, P_s, P_t, Polyakov) into 4 doubles of device memory:
    a torch float64 CUDA tensor (its first 4 elements) or a raw address."""
    ptr = dev_out.data_ptr() if hasattr(dev_out, "data_ptr") else int(dev_out)
    _check(load().su2_measure_device(ctypes.c_void_p(ptr)))


def su2_sweep_measure(n, every=1):
    m = int(n) // int(every) if every > 0 else 0
    hist = np.zeros((max(m, 1), 3))
    _check(load().su2_sweep_measure(int(n), int(every), _ptr(hist, ctypes.c_double)))
    return hist[:m]


def su2_links():
    """Links as float32 [V, 4, 4] (site lex, direction, component)."""
    dims = _keep.get("dims")
    if dims is None:
        raise Su2Error(SU2_ESTATE, "no lattice")
    V = int(np.prod(dims))
    out = np.empty((V, 4, 4), dtype=np.float32)
    _check(load().su2_links(_ptr(out, ctypes.c_float), out.size))
    return out


def su2_set_links(U, sweep_index):
    U = np.ascontiguousarray(U, dtype=np.float32)
    _check(load().su2_set_links(_ptr(U, ctypes.c_float), U.size, ctypes.c_uint64(sweep_index)))


def su2_sweep_index():
    out = ctypes.c_uint64(0)
    _check(load().su2_sweep_index(ctypes.byref(out)))
    return out.value


def su2_counters():
    """(heat-bath attempts, cap failures, learned proposals, accepted ones)."""
    out = np.zeros(4, dtype=np.uint64)
    _check(load().su2_counters(_ptr(out, ctypes.c_uint64)))
    return tuple(int(v) for v in out)


def su2_set_stream(stream=None):
    """stream: a torch.cuda.Stream, a raw hipStream_t integer, or None."""
    ptr = 0
    if stream is not None:
        ptr = getattr(stream, "cuda_stream", stream)
        _keep["stream"] = stream
    _check(load().su2_set_stream(ctypes.c_void_p(int(ptr)) if ptr else None))


def su2_set_plan(order_kind, lds_bytes):
    _check(load().su2_set_plan(int(order_kind), int(lds_bytes)))


def su2_tune(reps=2):
    """Time the pass-kernel launch plans and install the fastest; returns
    (order_kind, lds_bytes)."""
    out = (ctypes.c_int32 * 2)()
    _check(load().su2_tune(int(reps), out))
    return int(out[0]), int(out[1])


def su2_philox(seed, counters):
    c = np.ascontiguousarray(np.asarray(counters, dtype=np.uint32).reshape(-1, 4))
    out = np.zeros_like(c)
    _check(load().su2_philox(ctypes.c_uint64(seed), _ptr(c, ctypes.c_uint32), len(c),
                             _ptr(out, ctypes.c_uint32)))
    return out


def su2_synchronize():
    _check(load().su2_synchronize())


def su2_last_error():
    return load().su2_last_error().decode()


def su2_finalize():
    load().su2_finalize()
    _keep.pop("links", None)
    _keep.pop("dims", None)


# ---- batched replicas --------------------------------------------------------
_batch = {}


def _bcheck(rc):
    if rc != SU2_OK:
        raise Su2Error(rc, _lib.su2_batch_last_error().decode())
    return rc


def su2_batch_init(dims_list, betas, seeds, start):
    lib = load()
    d = np.ascontiguousarray(np.asarray(dims_list, dtype=np.int32).reshape(-1, 4))
    b = np.ascontiguousarray(np.asarray(betas, dtype=np.float64))
    sd = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
    if not (len(d) == len(b) == len(sd)):
        raise ValueError("dims, betas and seeds must have one entry per replica")
    _bcheck(lib.su2_batch_init(len(d), _ptr(d, ctypes.c_int32), _ptr(b, ctypes.c_double),
                               _ptr(sd, ctypes.c_uint64), int(start)))
    _batch["dims"] = [tuple(int(v) for v in row) for row in d]


def su2_batch_sweep(n=1):
    _bcheck(load().su2_batch_sweep(int(n)))


def su2_batch_set_mode(mode, tiles_per_item=1, lds_bytes=0):
    _bcheck(load().su2_batch_set_mode(int(mode), int(tiles_per_item), int(lds_bytes)))


def su2_batch_tune(sweeps=2):
    out = (ctypes.c_int32 * 3)()
    _bcheck(load().su2_batch_tune(int(sweeps), out))
    return int(out[0]), int(out[1]), int(out[2])


def su2_batch_set_spin_limit(ticks):
    _bcheck(load().su2_batch_set_spin_limit(ctypes.c_uint64(int(ticks))))


def su2_batch_plaquette():
    n = len(_batch.get("dims", []))
    out = np.zeros((max(n, 1), 3))
    _bcheck(load().su2_batch_plaquette(_ptr(out, ctypes.c_double)))
    return out[:n]


def su2_batch_links(r):
    if not 0 <= int(r) < len(_batch.get("dims", [])):
        raise Su2Error(SU2_EINVAL, f"no replica {r}")
    dims = _batch["dims"][r]
    V = int(np.prod(dims))
    out = np.empty((V, 4, 4), dtype=np.float32)
    _bcheck(load().su2_batch_links(int(r), _ptr(out, ctypes.c_float), out.size))
    return out


def su2_batch_counters(r):
    out = np.zeros(2, dtype=np.uint64)
    _bcheck(load().su2_batch_counters(int(r), _ptr(out, ctypes.c_uint64)))
    return int(out[0]), int(out[1])


def su2_batch_sweep_index():
    out = ctypes.c_uint64(0)
    _bcheck(load().su2_batch_sweep_index(ctypes.byref(out)))
    return out.value


def su2_batch_finalize():
    load().su2_batch_finalize()
    _batch.clear()


# ---- learned proposal ---------------------------------------------------------
NPARAM = 6433


def _mcheck(rc):
    if rc != SU2_OK:
        raise Su2Error(rc, _lib.su2_mlp_last_error().decode())
    return rc


def su2_cdf_knots(alphas):
    a = np.ascontiguousarray(np.asarray(alphas, dtype=np.float64))
    out = np.zeros((len(a), 33))
    _mcheck(load().su2_cdf_knots(_ptr(a, ctypes.c_double), len(a), _ptr(out, ctypes.c_double)))
    return out


def su2_mlp_set_params(params):
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
    _mcheck(load().su2_mlp_set_params(_ptr(p, ctypes.c_float), p.size))


def su2_mlp_get_params():
    m = np.zeros(NPARAM, dtype=np.float32)
    b = np.zeros(NPARAM, dtype=np.uint16)
    _mcheck(load().su2_mlp_get_params(_ptr(m, ctypes.c_float), _ptr(b, ctypes.c_uint16), NPARAM))
    return m, b


def su2_mlp_forward(alphas):
    a = np.ascontiguousarray(np.asarray(alphas, dtype=np.float32))
    out = np.zeros((len(a), 33), dtype=np.float32)
    _mcheck(load().su2_mlp_forward(_ptr(a, ctypes.c_float), len(a), _ptr(out, ctypes.c_float)))
    return out


def su2_mlp_loss_grad(alphas, target_logw):
    a = np.ascontiguousarray(np.asarray(alphas, dtype=np.float32))
    t = np.ascontiguousarray(np.asarray(target_logw, dtype=np.float32))
    loss = ctypes.c_float(np.nan)
    g = np.zeros(NPARAM, dtype=np.float32)
    _mcheck(load().su2_mlp_loss_grad(_ptr(a, ctypes.c_float), _ptr(t, ctypes.c_float), len(a),
                                     ctypes.byref(loss), _ptr(g, ctypes.c_float)))
    return loss.value, g


def su2_mlp_train(alphas, steps, lr0=3e-3, lr_min=1e-5):
    a = np.ascontiguousarray(np.asarray(alphas, dtype=np.float64))
    hist = np.zeros(max(int(steps), 1), dtype=np.float32)
    _mcheck(load().su2_mlp_train(_ptr(a, ctypes.c_double), len(a), int(steps), float(lr0),
                                 float(lr_min), _ptr(hist, ctypes.c_float)))
    return hist[:int(steps)]


def su2_mlp_tabulate(points=4096):
    _mcheck(load().su2_mlp_tabulate(int(points)))
    _keep["table_points"] = int(points)


def su2_cdf_tabulate(points=31):
    """The knot table from the integrated CDF instead of the network."""
    _mcheck(load().su2_cdf_tabulate(int(points)))
    _keep["table_points"] = int(points)


def su2_mlp_table():
    G = _keep["table_points"]
    out = np.zeros((G, 33), dtype=np.float32)
    _mcheck(load().su2_mlp_table(_ptr(out, ctypes.c_float), out.size))
    return out


def su2_set_proposal(kind, bf16_weights=None):
    """0 = heat-bath, 1 = learned proposal (from the current knot table, or
    from bf16_weights: 6433 BF16 bit patterns as uint16)."""
    if bf16_weights is None:
        _check(load().su2_set_proposal(int(kind), None, 0))
        return
    w = np.ascontiguousarray(np.asarray(bf16_weights, dtype=np.uint16))
    _check(load().su2_set_proposal(int(kind), _ptr(w, ctypes.c_uint16), w.size))
    if int(kind) == 1:
        _keep.setdefault("table_points", 31)


def su2_set_creutz(alpha_below=CREUTZ_SWITCH):
    """Heat-bath updates with alpha below alpha_below draw Creutz's way (0 = off)."""
    _check(load().su2_set_creutz(float(alpha_below)))


def su2_set_wide_offsets(on=True):
    """64-bit element offsets in the pass kernels even on a small lattice."""
    _check(load().su2_set_wide_offsets(1 if on else 0))


def su2_imh_counters():
    out = np.zeros(2, dtype=np.uint64)
    _check(load().su2_imh_counters(_ptr(out, ctypes.c_uint64)))
    return int(out[0]), int(out[1])
