"""Pins the oracle's Philox-4x32-10 and uniform mapping.

Philox is pinned against two third-party implementations of the published
generator (PyTorch's ATen header and rocRAND's header, both compiled for the
host at test time).  The uniform map is pinned by its definition at the ends.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "philox_libref.cpp")


def _cases():
    rng = np.random.default_rng(20090317)
    cases = [
        (0, 0, 0, 0, 0, 0),
        (1, 0, 0, 0, 0, 0),
        (0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF),
        (1, 0, 12345, 3 | (2 << 8), 999, 7),   # (site, mu|purpose<<8, sweep, slot)
        (0xDEADBEEF, 0x12345678, 16777215, 1, 199, 8),
    ]
    for _ in range(60):
        k = rng.integers(0, 2**32, size=2, dtype=np.uint64)
        c = rng.integers(0, 2**32, size=4, dtype=np.uint64)
        c[1] &= 0x3FFFFFFF  # rocRAND's 64-bit offset counts 32-bit outputs
        cases.append(tuple(int(v) for v in (*k, *c)))
    return cases


def _run_ref(tmp_path, which):
    exe = str(tmp_path / f"philox_{which}")
    if which == "aten":
        import torch
        inc = os.path.join(os.path.dirname(torch.__file__), "include")
        cmd = ["g++", "-O1", "-std=c++17", "-DUSE_ATEN", "-I", inc, SRC, "-o", exe]
    else:
        hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
        if not os.path.exists(hipcc):
            pytest.skip("hipcc not available")
        cmd = [hipcc, "-O1", "-DUSE_ROCRAND", SRC, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    cases = _cases()
    inp = "\n".join(" ".join(str(v) for v in c) for c in cases) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    words = np.array([[int(t) for t in line.split()] for line in out.strip().splitlines()],
                     dtype=np.uint64)
    return cases, words


@pytest.mark.parametrize("which", ["aten", "rocrand"])
def test_philox_matches_library(tmp_path, which):
    cases, ref = _run_ref(tmp_path, which)
    assert ref.shape == (len(cases), 4)
    for case, r in zip(cases, ref):
        k0, k1, c0, c1, c2, c3 = case
        got = oracle.philox4x32_10([c0, c1, c2, c3], [k0, k1])
        assert [int(v) for v in got] == [int(v) for v in r], case


def test_uniform_map_ends_and_exactness():
    # u = ((w >> 8) + 1) * 2^-24 lies in (0, 1]
    assert oracle.uniform(0) == 2.0 ** -24
    assert oracle.uniform(0xFF) == 2.0 ** -24
    assert oracle.uniform(0x100) == 2.0 * 2.0 ** -24
    assert oracle.uniform(0xFFFFFFFF) == 1.0
    rng = np.random.default_rng(5)
    for w in rng.integers(0, 2**32, size=200, dtype=np.uint64):
        u = oracle.uniform(int(w))
        assert np.float32(u) == u  # exactly representable in FP32
        assert u == ((int(w) >> 8) + 1) / 2.0 ** 24


def test_philox_counter_sensitivity():
    """Every counter word and key word changes the block (no aliasing in the
    layout site / mu|purpose / sweep / slot)."""
    base = oracle.philox4x32_10([7, 2, 3, 4], [11, 13])
    for i in range(4):
        c = [7, 2, 3, 4]
        c[i] += 1
        assert not np.array_equal(oracle.philox4x32_10(c, [11, 13]), base)
    for i in range(2):
        k = [11, 13]
        k[i] += 1
        assert not np.array_equal(oracle.philox4x32_10([7, 2, 3, 4], k), base)
