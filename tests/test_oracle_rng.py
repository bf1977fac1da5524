"""Pins of the oracle's random numbers (reading R13: Philox4x32-10, 23-bit
uniforms, Box-Muller normals; section 3.4 asks for Gaussian increments).

Philox is pinned bitwise against rocRAND's open-source engine header (an
independent implementation), compiled host-only here.  Uniforms are pinned
by exact values and exact binary32 representability; Box-Muller by its
defining identities and by moments / a KS test of many normals."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.stats

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    exe = str(tmp_path_factory.mktemp("rr") / "rr")
    subprocess.run([hipcc, "--offload-host-only", "-x", "hip", "-O1", "-o", exe,
                    os.path.join(HERE, "rocrand_philox_ref.cpp")], check=True)

    def run(rows):
        inp = "".join("%d %d %d %d %d %d\n" % tuple(r) for r in rows)
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
        return [[int(v) for v in ln.split()] for ln in out.strip().splitlines()]
    return run


def test_philox_matches_rocrand(oracle_lib, rocrand_ref):
    rng = np.random.default_rng(1234)
    rows = [[0, 0, 0, 0, 0, 0], [1, 0, 0, 0, 0, 0], [0, 0, 0, 0, 1, 0], [0, 0, 0, 0, 0, 1]]
    for _ in range(300):
        c = rng.integers(0, 2 ** 32, size=4, dtype=np.uint64)
        c[1] %= 2 ** 29        # keeps 4*(c0 + 2^32 c1) inside rocRAND's 64-bit offset
        k = rng.integers(0, 2 ** 32, size=2, dtype=np.uint64)
        rows.append([int(v) for v in c] + [int(v) for v in k])
    # counters of the form the estimator uses: (block, path, node, I<<16|S)
    for (m, p, node, inst, step) in [(0, 0, 0, 0, 0), (374, 99_999, 752, 3, 7), (0x7FFFFFFF, 5, 31, 65535, 65535)]:
        rows.append([m, p, node, (inst << 16) | step, 0, 0])
        rows.append([m, p, node, (inst << 16) | step, 0xDEADBEEF, 0x12345678])
    ref = rocrand_ref(rows)
    assert len(ref) == len(rows)
    for r, want in zip(rows, ref):
        got = oracle_lib.philox4x32_10(r[:4], r[4:])
        assert got == want, (r, got, want)


def test_philox_sensitivity(oracle_lib):
    # every counter and key word matters (a dropped word would collide)
    base = oracle_lib.philox4x32_10([1, 2, 3, 4], [5, 6])
    for w in range(6):
        ctr, key = [1, 2, 3, 4], [5, 6]
        if w < 4:
            ctr[w] ^= 1
        else:
            key[w - 4] ^= 1
        assert oracle_lib.philox4x32_10(ctr, key) != base


def test_uniform_exact_values(oracle_lib):
    assert oracle_lib.uniform(0) == 2.0 ** -24
    assert oracle_lib.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert oracle_lib.uniform(0x80000000) == 0.5 + 2.0 ** -24
    rng = np.random.default_rng(7)
    for r in rng.integers(0, 2 ** 32, size=2000, dtype=np.uint64):
        u = oracle_lib.uniform(int(r))
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u          # exact in binary32 too
        assert u == ((int(r) >> 9) * 2 + 1) * 2.0 ** -24


def test_box_muller_identities(oracle_lib):
    rng = np.random.default_rng(8)
    for r0, r1 in rng.integers(0, 2 ** 32, size=(500, 2), dtype=np.uint64):
        n1, n2 = oracle_lib.box_muller(int(r0), int(r1))
        u0, u1 = oracle_lib.uniform(int(r0)), oracle_lib.uniform(int(r1))
        assert abs((n1 * n1 + n2 * n2) - (-2.0 * math.log(u0))) < 1e-12 * max(1.0, -2.0 * math.log(u0))
        ang = math.atan2(n2, n1) % (2 * math.pi)
        assert abs(ang - 2 * math.pi * u1) < 1e-9 or abs(abs(ang - 2 * math.pi * u1) - 2 * math.pi) < 1e-9


def test_stream_layout(oracle_lib):
    """Stream word q of a path is word q mod 4 of the Philox block with
    counter (q div 4, path, node, I<<16 | S); substep k takes words 3k,
    3k+1 for Box-Muller and word 3k+2 for the bridge uniform."""
    P = oracle_lib.Problem(n_xi=33, n_eta=33, sub_xi=2, sub_eta=1, seed=0x0123456789ABCDEF,
                           instance_id=9, mesh_step=4)
    key = [0x89ABCDEF, 0x01234567]

    def word(node, path, q):
        return oracle_lib.philox4x32_10([q // 4, path, node, (9 << 16) | 4], key)[q % 4]
    for (node, path, k) in [(0, 0, 0), (3, 17, 1), (3, 17, 2), (3, 17, 3), (30, 9999, 498), (30, 9999, 499)]:
        for q in (3 * k, 3 * k + 1, 3 * k + 2):
            assert oracle_lib.stream_word(P, node, path, q) == word(node, path, q)
        want = oracle_lib.box_muller(word(node, path, 3 * k), word(node, path, 3 * k + 1))
        assert oracle_lib.normals(P, node, path, k) == want
        assert oracle_lib.bridge_uniform(P, node, path, k) == oracle_lib.uniform(word(node, path, 3 * k + 2))
    # mesh step uses only its low 16 bits; instance id sits above it
    P2 = oracle_lib.Problem(n_xi=33, n_eta=33, sub_xi=2, sub_eta=1, seed=0x0123456789ABCDEF,
                            instance_id=9, mesh_step=4 + 65536)
    assert oracle_lib.stream_word(P2, 1, 2, 3) == oracle_lib.stream_word(P, 1, 2, 3)


def test_normals_distribution(oracle_lib):
    """Normals of one stream: mean 0, variance 1, KS against N(0,1), and
    no correlation between the pair members or between substeps."""
    P = oracle_lib.Problem(n_xi=33, n_eta=33, sub_xi=2, sub_eta=1, seed=42)
    a = np.array([oracle_lib.normals(P, 3, p, k) for p in range(200) for k in range(100)])
    n = a.size
    x = a.ravel()
    assert abs(x.mean()) < 4.0 / math.sqrt(n)
    assert abs(x.var() - 1.0) < 4.0 * math.sqrt(2.0 / n)
    assert scipy.stats.kstest(x, "norm").pvalue > 1e-4
    c = np.corrcoef(a[:, 0], a[:, 1])[0, 1]
    assert abs(c) < 4.0 / math.sqrt(len(a))
    c2 = np.corrcoef(a[:-1, 0], a[1:, 0])[0, 1]
    assert abs(c2) < 4.0 / math.sqrt(len(a))
    u = np.array([oracle_lib.bridge_uniform(P, 3, p, k) for p in range(100) for k in range(100)])
    assert scipy.stats.kstest(u, "uniform").pvalue > 1e-4
