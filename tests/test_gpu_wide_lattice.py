"""The largest lattices: 2^29 sites (128 x 128 x 128 x 256, 32 GiB of FP32
links), the size from which the link arrays pass 4 GiB and the kernels take
64-bit element offsets by themselves, and 2^31 sites (256^3 x 128, 128 GiB),
where site indices pass the signed 32-bit range (the Philox counter allows up
to 2^32 sites).  The oracle cannot form such a lattice,
so it checks sampled links: an update it recomputes reads only the links it
is given -- the 18 staple inputs of Eq. (6) and the link itself, gathered
from the GPU's own field -- which sit in an FP64 field of the full size held
in lazily mapped memory (only the pages written take host memory).

Bars as in the other parity tests: hot-start links <= 1e-6; updated links
the per-link conditioned bar, with decision flips counted; unitarity
<= 1e-6; links a pass does not own bit-identical.
"""
import mmap

import numpy as np
import pytest

import oracle
from parity import UNIT_TOL, compare_links_conditioned, staple_inputs, unitarity_error

pytestmark = pytest.mark.gpu

SIZES = [(128, 128, 128, 256), (256, 256, 256, 128)]
BETA, SEED = 2.4, 5


class Geo:
    def __init__(self, dims):
        self.dims = dims
        self.V = int(np.prod(dims))
        self.half = self.V // 2


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_0903_3053_amd import su2
    su2.load()
    yield su2
    su2.su2_finalize()


@pytest.fixture(scope="module", params=SIZES, ids=["2^29", "2^31"])
def geo(request):
    return Geo(request.param)


@pytest.fixture(scope="module")
def links(lib, geo):
    """The caller-owned device field every test of this size re-initialises."""
    import torch
    need = 64 * geo.V
    free, _ = torch.cuda.mem_get_info()
    if free < need + (8 << 30):
        pytest.skip(f"needs {(need >> 30) + 8} GiB of free GPU memory, {free >> 30} GiB free")
    buf = torch.empty(16 * geo.V, dtype=torch.float32, device="cuda")
    buf.geo = geo
    yield buf
    lib.su2_finalize()
    del buf
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def field(geo):
    """float64 [V, 4, 4] of zeros in anonymous memory without huge pages (only
    address space until written; a host that refuses that much is skipped)."""
    try:
        mem = mmap.mmap(-1, geo.V * 16 * 8, flags=mmap.MAP_PRIVATE)
    except (OSError, MemoryError) as e:
        pytest.skip(f"cannot map {geo.V * 128 >> 30} GiB of address space: {e}")
    if hasattr(mmap, "MADV_NOHUGEPAGE"):
        mem.madvise(mmap.MADV_NOHUGEPAGE)
    yield np.frombuffer(mem, dtype=np.float64).reshape(geo.V, 4, 4)


def init(lib, buf, start):
    lib.su2_init_ex(buf.geo.dims, BETA, SEED, start, buf.data_ptr(), buf.numel() * 4)


def parity(geo, lex):
    lex = np.asarray(lex, dtype=np.int64)
    L0, L1, L2 = geo.dims[:3]
    return (lex % L0 + (lex // L0) % L1 + (lex // (L0 * L1)) % L2 + lex // (L0 * L1 * L2)) % 2


def gather(buf, lex, mu):
    """Links U_mu(lex) (broadcast shapes) from the device field, float64
    [..., 4]: array 2 mu + parity, element lex / 2 (the su2_init_ex layout)."""
    import torch
    geo = buf.geo
    lex, mu = np.broadcast_arrays(np.asarray(lex, dtype=np.int64), np.asarray(mu, dtype=np.int64))
    el = (2 * mu + parity(geo, lex)) * geo.half + lex // 2
    idx = torch.from_numpy(np.ascontiguousarray(el.ravel())).to(buf.device)
    return buf.view(-1, 4)[idx].double().cpu().numpy().reshape(lex.shape + (4,))


def sample_sites(geo, rng, n, p=None):
    """n random sites plus the corners of the lattice (first and last sites,
    the last time slice, the middle), all of parity p if given (x0 moved by
    one where needed)."""
    V = geo.V
    slab = geo.dims[0] * geo.dims[1] * geo.dims[2]
    corners = [0, 1, V - 2, V - 1, V - slab, V - slab + 3, slab - 1, V // 2 - 1, V // 2]
    lex = np.concatenate([rng.integers(0, V, size=n, dtype=np.int64), corners])
    if p is not None:
        lex = np.where(parity(geo, lex) == p, lex, lex ^ 1)
    return np.unique(lex)


def neighbourhood(geo, sites, mu):
    """(lex, direction) of every link the update of U_mu at the sites reads:
    the 18 staple inputs and the link itself."""
    src, dirs = staple_inputs(geo.dims, sites, mu)
    return (np.concatenate([src.ravel(), sites]),
            np.concatenate([dirs.ravel(), np.full(len(sites), mu)]))


def test_hot_start_sampled(lib, links):
    geo = links.geo
    init(lib, links, lib.HOT)
    sites = sample_sites(geo, np.random.default_rng(1), 600)
    got = gather(links, sites[:, None], np.arange(4)[None, :])
    ref = oracle.init_sites(geo.dims, SEED, 1, sites)
    assert np.max(np.abs(got - ref)) <= 1e-6
    assert unitarity_error(got) <= UNIT_TOL
    # Haar links: 1/2 Tr of a plaquette or of a Polyakov loop has mean 0 and
    # standard deviation 1/2, so their averages over 6 V plaquettes and over
    # the spatial sites are 0 to well within these bars
    P = lib.su2_plaquette_st()
    L = lib.su2_polyakov()
    print(f"{geo.dims}, hot start: P = {P[0]:.2e} (P_s {P[1]:.2e}, P_t {P[2]:.2e}), L = {L:.2e}")
    assert np.max(np.abs(P)) < 1e-4 and abs(L) < 2.5e-3


def test_first_pass_from_the_oracles_hot_start(lib, links, field):
    """The first pass of sweep 0 from the hot start: every input of the
    sampled updates is the oracle's own hot-start link (oracle_init_sites),
    none is read from the GPU."""
    geo = links.geo
    init(lib, links, lib.HOT)
    lib.su2_set_plan(1108, 32768)
    p, mu = 1, 0
    sites = sample_sites(geo, np.random.default_rng(5), 250, p)
    all_lex, all_mu = neighbourhood(geo, sites, mu)
    lex_u = np.unique(all_lex)
    field[lex_u] = oracle.init_sites(geo.dims, SEED, 1, lex_u)
    lib.su2_pass(p, mu)
    new = gather(links, sites, mu)
    out, tries, margin = oracle.update_sites(geo.dims, field, BETA, SEED, 0, mu, sites)
    w = np.array([oracle.staple(geo.dims, field, int(x), mu) for x in sites])
    k = np.sqrt(np.sum(w * w, axis=1))
    x0 = np.where(tries <= 7, np.sum(out * w, axis=1) / k, np.nan)
    st = compare_links_conditioned(new, out, margin, k, x0)
    print(f"{geo.dims}, first pass from the oracle's hot start: {st['n']} sampled updates, {st['flips']} flips, "
          f"max err {st['max_err_rest']:.2e}")
    assert st["unexplained"] == 0 and st["flips"] <= 2
    assert unitarity_error(new) <= UNIT_TOL


def test_sweep_pass_by_pass_sampled(lib, links, field):
    """Two sweeps from the hot start with the benchmark's launch plan (tile
    order 1108, 32 KiB LDS), then each pass of the third sweep on its own:
    sampled updated links against the oracle's update of the same inputs."""
    geo = links.geo
    init(lib, links, lib.HOT)
    lib.su2_set_plan(1108, 32768)
    lib.su2_sweep(2)
    s = lib.su2_sweep_index()
    rng = np.random.default_rng(2)
    n_upd = flips = 0
    worst = 0.0
    for p in (1, 0):
        for mu in range(4):
            sites = sample_sites(geo, rng, 250, p)
            all_lex, all_mu = neighbourhood(geo, sites, mu)
            before = gather(links, all_lex, all_mu)
            field[all_lex, all_mu] = before
            lib.su2_pass(p, mu)
            after = gather(links, all_lex, all_mu)
            owned = (all_mu == mu) & (parity(geo, all_lex) == p)
            assert np.array_equal(after[~owned], before[~owned]), (p, mu)
            new = gather(links, sites, mu)
            out, tries, margin = oracle.update_sites(geo.dims, field, BETA, SEED, s, mu, sites)
            w = np.array([oracle.staple(geo.dims, field, int(x), mu) for x in sites])
            k = np.sqrt(np.sum(w * w, axis=1))
            x0 = np.where(tries <= 7, np.sum(out * w, axis=1) / k, np.nan)
            st = compare_links_conditioned(new, out, margin, k, x0)
            assert st["unexplained"] == 0, (p, mu, st)
            assert unitarity_error(new) <= UNIT_TOL
            n_upd += len(sites)
            flips += st["flips"]
            worst = max(worst, st["max_err_rest"])
    print(f"{geo.dims}, sweep {s} pass by pass: {n_upd} sampled updates, {flips} flipped "
          f"decisions, max err {worst:.2e}")
    assert flips <= 2
    assert lib.su2_sweep_index() == s


def test_overrelax_pass_sampled(lib, links, field):
    """One overrelaxation pass: sampled links become V U^dag V (V = w/|w|)
    from the oracle's staple of the same inputs."""
    geo = links.geo
    init(lib, links, lib.HOT)
    lib.su2_set_plan(1108, 32768)
    lib.su2_sweep(1)
    p, mu = 0, 2
    sites = sample_sites(geo, np.random.default_rng(3), 250, p)
    all_lex, all_mu = neighbourhood(geo, sites, mu)
    field[all_lex, all_mu] = gather(links, all_lex, all_mu)
    lib.su2_overrelax_pass(p, mu)
    new = gather(links, sites, mu)
    ref = np.zeros_like(new)
    for i, x in enumerate(sites):
        w = oracle.staple(geo.dims, field, int(x), mu)
        Vq = w / np.sqrt(np.sum(w * w))
        u = field[x, mu] * np.array([1.0, -1.0, -1.0, -1.0])
        ref[i] = oracle.qmul(oracle.qmul(Vq, u), Vq)
    assert np.max(np.abs(new - ref)) <= 1e-5
    assert unitarity_error(new) <= UNIT_TOL


def test_plans_agree_at_full_size(lib, links):
    """Two measured sweeps from the hot start with the benchmark's plan, the
    fused pairs and the identity tile order: sampled links and the counters
    bit-identical, the in-sweep plaquettes equal to 1e-13, and the in-sweep
    plaquette equal to the plaquette kernel's on the same links."""
    geo = links.geo
    sites = sample_sites(geo, np.random.default_rng(4), 4000)
    res = []
    for plan in ((1108, 32768), (lib.FUSED_PAIRS, 0), (0, 0)):
        init(lib, links, lib.HOT)
        lib.su2_set_plan(*plan)
        hist = lib.su2_sweep_measure(2, 1)
        fused = lib.su2_plaquette_st()
        lib.su2_set_plan(*plan)  # discards the in-sweep partials
        direct = lib.su2_plaquette_st()
        assert np.max(np.abs(fused - direct)) <= 2e-6, plan
        np.testing.assert_allclose(fused, hist[-1], rtol=0, atol=1e-13)
        res.append((gather(links, sites[:, None], np.arange(4)[None, :]), lib.su2_counters(), hist))
    print(f"{geo.dims}, beta {BETA}: P after 2 sweeps {res[0][2][-1]}")
    for got, counters, hist in res[1:]:
        assert np.array_equal(got, res[0][0])
        assert counters == res[0][1]
        np.testing.assert_allclose(hist, res[0][2], rtol=0, atol=1e-13)
    assert unitarity_error(res[0][0]) <= UNIT_TOL
