"""The C-ABI library builds, loads and exports every entry point include/*.h
declares; argument and state errors come back as codes without device work
(runs without a GPU)."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b((?:su2|ising)_\w+)\s*\(", text))
    return names


@pytest.fixture(scope="module")
def lib():
    from paper_0903_3053_amd import su2
    if not os.path.exists(su2.LIBPATH):
        from paper_0903_3053_amd import build
        build.build()
    return su2.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert {"su2_init", "su2_sweep", "su2_plaquette", "su2_links"} <= names
    for n in sorted(names):
        assert hasattr(lib, n), n


def test_binding_lists_every_declared_symbol():
    from paper_0903_3053_amd import ising, su2
    assert _declared() == set(su2.EXPORTS) | set(ising.EXPORTS)


def test_ising_errors_without_device_work(lib):
    from paper_0903_3053_amd import ising, su2
    lib = ising.load()
    lib.ising_finalize()
    assert lib.ising_sweep(1) == su2.SU2_ESTATE
    out = (ctypes.c_double * 2)()
    assert lib.ising_observables(out) == su2.SU2_ESTATE
    assert b"ising_init" in lib.ising_last_error()
    for dims, beta, start in [((3, 4), 0.4, 0), ((4, 0), 0.4, 0), ((4, 4), -1.0, 0),
                              ((4, 4), float("inf"), 0), ((4, 4), 0.4, 2)]:
        d = np.asarray(dims, dtype=np.int32)
        assert lib.ising_init(d.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), beta, 1, start) == su2.SU2_EINVAL
    assert lib.ising_init(None, 0.4, 1, 0) == su2.SU2_EINVAL
    lay = ctypes.c_int32(-1)
    assert lib.ising_layout(ctypes.byref(lay)) == su2.SU2_ESTATE
    for dims, layout in [((96, 4), ising.LAYOUT_BITS), ((64, 4), 3), ((64, 4), -1)]:
        d = np.asarray(dims, dtype=np.int32)
        assert lib.ising_init_ex(d.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 0.4, 1, 0,
                                 layout) == su2.SU2_EINVAL


def test_state_errors_before_init(lib):
    from paper_0903_3053_amd import su2
    lib.su2_finalize()
    assert lib.su2_sweep(1) == su2.SU2_ESTATE
    assert lib.su2_pass(0, 0) == su2.SU2_ESTATE
    assert np.isnan(lib.su2_plaquette())
    out = (ctypes.c_uint64 * 4)()
    assert lib.su2_counters(out) == su2.SU2_ESTATE
    assert b"su2_init" in lib.su2_last_error()
    assert lib.su2_bind(ctypes.c_void_p(4096), 1 << 20) == su2.SU2_ESTATE
    w = np.zeros(6433, dtype=np.uint16)
    wp = w.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16))
    assert lib.su2_set_proposal(1, wp, 6433) == su2.SU2_ESTATE
    assert lib.su2_set_proposal(0, None, 0) == su2.SU2_ESTATE
    assert lib.su2_philox(1, None, 3, None) == su2.SU2_EINVAL
    assert lib.su2_polyakov_correlator_noalloc(1, ctypes.c_void_p(4096)) == su2.SU2_ESTATE


@pytest.mark.parametrize("dims,beta,start", [
    ((3, 4, 4, 4), 2.3, 0),      # odd extent
    ((4, 4, 0, 4), 2.3, 0),      # zero extent
    ((4, 4, 4, -2), 2.3, 0),     # negative extent
    ((4, 4, 4, 4), -1.0, 0),     # negative beta
    ((4, 4, 4, 4), float("nan"), 0),
    ((4, 4, 4, 4), float("inf"), 1),
    ((4, 4, 4, 4), 2.3, 2),      # bad start
    ((65536, 65536, 2, 2), 2.3, 0),  # volume 2^34
])
def test_init_rejects_bad_arguments(lib, dims, beta, start):
    from paper_0903_3053_amd import su2
    d = (ctypes.c_int32 * 4)(*dims)
    assert lib.su2_init(d, beta, 1, start) == su2.SU2_EINVAL
    assert len(lib.su2_last_error()) > 0


def test_python_binding_raises(lib):
    from paper_0903_3053_amd import su2
    with pytest.raises(su2.Su2Error):
        su2.su2_init((5, 4, 4, 4), 2.3, 1, 0, torch_memory=False)


def test_extension_entry_points_reject_bad_arguments(lib):
    """The batched-replica and learned-proposal entry points check their
    arguments and state before any device work."""
    from paper_0903_3053_amd import su2
    i32, f64, u64 = ctypes.c_int32, ctypes.c_double, ctypes.c_uint64
    # batch: count, extents, coupling, start; calls before a batch exists
    dims = (i32 * 4)(3, 4, 4, 4)
    betas = (f64 * 1)(2.0)
    seeds = (u64 * 1)(1)
    assert lib.su2_batch_init(0, dims, betas, seeds, 1) == su2.SU2_EINVAL
    assert lib.su2_batch_init(1, dims, betas, seeds, 1) == su2.SU2_EINVAL  # odd extent
    dims_ok = (i32 * 4)(4, 4, 4, 4)
    assert lib.su2_batch_init(1, dims_ok, (f64 * 1)(-1.0), seeds, 1) == su2.SU2_EINVAL
    assert lib.su2_batch_init(1, dims_ok, betas, seeds, 7) == su2.SU2_EINVAL
    assert lib.su2_batch_init(1, None, betas, seeds, 1) == su2.SU2_EINVAL
    assert lib.su2_batch_sweep(1) == su2.SU2_ESTATE
    assert lib.su2_batch_set_mode(0, 1, 0) == su2.SU2_ESTATE
    # learned proposal: parameter count, CDF arguments, calls before parameters exist
    p = np.zeros(6432, dtype=np.float32)
    assert lib.su2_mlp_set_params(p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), 6432) == su2.SU2_EINVAL
    a = (f64 * 2)(1.0, -1.0)
    k = (f64 * 66)()
    assert lib.su2_cdf_knots(a, 2, k) == su2.SU2_EINVAL  # negative alpha
    assert lib.su2_cdf_knots(a, -1, k) == su2.SU2_EINVAL
    assert lib.su2_cdf_knots(a, 0, k) == su2.SU2_OK
    af = (ctypes.c_float * 1)(1.0)
    kf = (ctypes.c_float * 33)()
    assert lib.su2_mlp_forward(af, 1, kf) == su2.SU2_ESTATE
    assert lib.su2_mlp_tabulate(31) == su2.SU2_ESTATE
    # the CDF table needs no parameters; its size is checked before any device call
    assert lib.su2_cdf_tabulate(1) == su2.SU2_EINVAL
    assert lib.su2_cdf_tabulate(65537) == su2.SU2_EINVAL
    # the lattice is gone after su2_finalize: proposal selection is a state error
    lib.su2_finalize()
    assert lib.su2_set_proposal(1, None, 0) == su2.SU2_ESTATE
    assert lib.su2_set_creutz(ctypes.c_double(1.0)) == su2.SU2_ESTATE
    assert lib.su2_set_wide_offsets(1) == su2.SU2_ESTATE
