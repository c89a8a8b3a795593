"""The no-allocation entry point su2_polyakov_correlator_noalloc against the
allocating su2_polyakov_correlator (same kernels, same order: bit-identical)
and against the oracle (FP32 ordered products vs FP64: <= 1e-6), on two
calls in a row of which the second has the smaller input; then the size
limit of its scratch."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_0903_3053_amd import su2
    su2.load()
    yield su2
    su2.su2_finalize()


def test_noalloc_correlator_matches_the_allocating_one(lib):
    import torch
    for dims, rmax in (((16, 16, 16, 8), 8), ((8, 6, 10, 4), 3)):
        lib.su2_init(dims, 2.3, 4, lib.HOT)
        lib.su2_sweep(3)
        ref = lib.su2_polyakov_correlator(rmax)
        out = torch.full((rmax + 2,), float("nan"), dtype=torch.float64, device="cuda")
        lib.su2_polyakov_correlator_noalloc(rmax, out)
        lib.su2_synchronize()
        got = out.cpu().numpy()
        want = oracle.polyakov_correlator(dims, lib.su2_links().astype(np.float64), rmax)
        print(f"no-alloc correlator {dims}, rmax {rmax}: max |diff| to the allocating call "
              f"{np.max(np.abs(got[:rmax + 1] - ref)):.1e}, to the oracle {np.max(np.abs(got[:rmax + 1] - want)):.1e}")
        np.testing.assert_array_equal(got[:rmax + 1], ref)
        assert np.isnan(got[rmax + 1])  # nothing written past rmax
        np.testing.assert_allclose(got[:rmax + 1], want, rtol=0, atol=1e-6)


def test_noalloc_correlator_rejects_what_does_not_fit(lib):
    import torch
    out = torch.zeros(64, dtype=torch.float64, device="cuda")
    lib.su2_init((96, 96, 96, 2), 2.3, 1, lib.COLD)  # 96^3 spatial sites > 2^19 doubles
    with pytest.raises(lib.Su2Error, match="scratch"):
        lib.su2_polyakov_correlator_noalloc(1, out)
    lib.su2_init((8, 8, 8, 4), 2.3, 1, lib.COLD)
    with pytest.raises(lib.Su2Error):
        lib.su2_polyakov_correlator_noalloc(5, out)  # rmax above L/2
    with pytest.raises(lib.Su2Error):
        lib.su2_polyakov_correlator_noalloc(2, out.data_ptr() + 4)  # misaligned
    lib.su2_polyakov_correlator_noalloc(4, out)
    lib.su2_synchronize()
    np.testing.assert_array_equal(out.cpu().numpy()[:5], np.ones(5))  # cold lattice: C = 1
