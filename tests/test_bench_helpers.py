"""The bench's host-side work counts, which the reported roofline divides by
measured time, checked against brute force over the block products of small
matrices: algorithmic flops (sum of 2 m n k), MFMA-issued flops (m, n and k
rounded up to 16), the no-reuse operand stream (8 (m k + k n) bytes per
product), block norms, and the work the norm-bound screen leaves."""
import math

import numpy as np
import pytest

import bench
from synth import banded_uneven, make_matrix, rng_of


def _blocks(M):
    """[(I, J, values)] of a host block-CSR matrix, in storage order."""
    out, off = [], 0
    data = np.asarray(M.data)
    for i in range(len(M.rbs)):
        for p in range(M.row_ptr[i], M.row_ptr[i + 1]):
            j = int(M.col_ind[p])
            n = int(M.rbs[i]) * int(M.cbs[j])
            out.append((i, j, data[off:off + n]))
            off += n
    return out


def _brute(A, B, alpha=1.0, eps=0.0):
    """Per-product counts and per-C-block norm bounds, by plain loops."""
    pad = lambda x: 16 * math.ceil(x / 16)
    brow = {}
    for k, j, v in _blocks(B):
        brow.setdefault(k, []).append((j, math.sqrt(sum(float(x) * float(x) for x in v))))
    per_c = {}
    for i, k, v in _blocks(A):
        na = math.sqrt(sum(float(x) * float(x) for x in v))
        m, kk = int(A.rbs[i]), int(A.cbs[k])
        for j, nb in brow.get(k, []):
            n = int(B.cbs[j])
            w = per_c.setdefault((i, j), [0, 0, 0, 0, 0.0])
            w[0] += 1
            w[1] += 2 * m * n * kk
            w[2] += 2 * pad(m) * pad(n) * pad(kk)
            w[3] += 8 * (m * kk + kk * n)
            w[4] += abs(alpha) * na * nb
    margin = max(1e-6, 4.0 * (sum(int(x) for x in A.cbs) + 4.0) * 2.0 ** -53)
    kept = {key: w for key, w in per_c.items() if not (w[4] * (1 + margin) < eps and w[4] < 1e150)}
    tot = lambda d, c: sum(w[c] for w in d.values())
    return {"all": [tot(per_c, c) for c in range(4)], "kept": [tot(kept, c) for c in range(4)],
            "screened": len(per_c) - len(kept)}


def _pair(seed):
    rng = rng_of(seed)
    m = rng.choice(np.array([1, 5, 13, 16, 17, 23, 32, 45], np.int32), 9)
    k = rng.choice(np.array([2, 7, 16, 29, 33], np.int32), 7)
    n = rng.choice(np.array([3, 13, 16, 31, 64], np.int32), 8)
    return make_matrix(rng, m, k, 0.5), make_matrix(rng, k, n, 0.5)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_flops_and_stream_match_brute_force(seed):
    A, B = _pair(seed)
    ref = _brute(A, B)
    F, issued = bench.mfma_padding(A, B)
    assert F == ref["all"][1]
    assert issued == ref["all"][2]
    assert bench.stream_bytes(A, B) == ref["all"][3]


@pytest.mark.parametrize("chunk", [1, 50, 1 << 26])
def test_block_norms(chunk):
    A, _ = _pair(4)
    want = [np.sqrt(np.sum(v.astype(np.float64) ** 2)) for _, _, v in _blocks(A)]
    np.testing.assert_allclose(bench.block_norms(A, chunk=chunk), want, rtol=1e-14, atol=0)


def test_screened_work_without_screen_is_all_work():
    A, B = _pair(5)
    ref = _brute(A, B)
    w = bench.screened_work(A, B, 1.0, 0.0)
    assert w["products_run"] == ref["all"][0]
    assert w["flops_run"] == ref["all"][1]
    assert w["issued_run"] == ref["all"][2]
    assert w["stream_run"] == ref["all"][3]
    assert w["screened_blocks"] == 0


@pytest.mark.parametrize("alpha,eps", [(1.0, 1e-10), (-3.0, 1e-6)])
def test_screened_work_matches_brute_force(alpha, eps):
    A, B = banded_uneven(seed=83, occupancy=0.3, target=700, decay=2.0)
    ref = _brute(A, B, alpha, eps)
    w = bench.screened_work(A, B, alpha, eps)
    assert ref["screened"] > 0 and ref["kept"][0] < ref["all"][0]
    assert w["screened_blocks"] == ref["screened"]
    assert w["products_run"] == ref["kept"][0]
    for key, c in (("flops_run", 1), ("issued_run", 2), ("stream_run", 3)):
        assert w[key] == pytest.approx(ref["kept"][c], rel=1e-12)
