"""Pins for the codebook part of the oracle (NN, k-means, qCH).

Sources of truth: the paper's own codebook-size figure (Sec. 5.1), SciPy's
independent vector quantizer and k-means (scipy.cluster.vq), the exact Chamfer
oracle (itself pinned to the paper's worked example) for codebooks that hold
every vector, closed forms, invariants, an error bound from the triangle and
Cauchy-Schwarz inequalities, and brute-force loops on tiny integer inputs.
"""
import warnings

import numpy as np
import pytest
from scipy.cluster import vq as scipy_vq

import oracle


def _unit(rng, n, d=128):
    x = rng.standard_normal((n, d))
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def _csr(lengths):
    o = np.zeros(len(lengths) + 1, np.int64)
    o[1:] = np.cumsum(lengths)
    return o


def _clustered(rng, n, k, d=128, spread=0.3):
    centers = _unit(rng, k, d)
    x = centers[rng.integers(0, k, n)] + spread * rng.standard_normal((n, d)) / np.sqrt(d)
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def test_codebook_size_rule_matches_paper():
    # Sec. 5.1 prints the rule's value for the 597M-vector collection: about 262k
    assert oracle.codebook_size(597_000_000) == 262_144
    # the 100k-document synthetic corpus (8,014,384 vectors): 16 sqrt(V) = 45,296 -> 2^15
    assert oracle.codebook_size(8_014_384) == 32_768
    # 72M vectors (the 1M-document corpus): 16 sqrt(V) = 135,760 -> 2^17
    assert oracle.codebook_size(71_998_246) == 131_072
    for n in [1, 2, 100, 12_345, 10 ** 9]:
        k = oracle.codebook_size(n)
        assert k & (k - 1) == 0 and k <= 16 * np.sqrt(n) < 2 * k


def test_nn_assign_matches_scipy_vq():
    rng = np.random.default_rng(0)
    x = _clustered(rng, 600, 20)
    C = _unit(rng, 37)
    codes = oracle.nn_assign(x, C)
    ref_codes, ref_dist = scipy_vq.vq(x, C)
    np.testing.assert_array_equal(codes, ref_codes)
    d2 = oracle.sq_distances(x, C)
    np.testing.assert_allclose(np.sqrt(d2[np.arange(600), codes]), ref_dist, rtol=1e-12)
    # the distance matrix against its expansion ||x||^2 - 2<x, c> + ||c||^2
    exp = (x * x).sum(1)[:, None] - 2 * x @ C.T + (C * C).sum(1)[None, :]
    np.testing.assert_allclose(d2, exp, atol=1e-12)


def test_nn_assign_ties_go_to_smallest_index():
    C = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 0.0], [0.0, 1.0]])
    x = np.array([[1.0, 0.0], [0.0, 1.0], [0.5, 0.5], [-1.0, 0.0]])
    np.testing.assert_array_equal(oracle.nn_assign(x, C), [0, 1, 0, 1])
    # [-1, 0] is sqrt(2) from both [0, 1] rows and 2 from both [1, 0] rows: index 1


@pytest.mark.parametrize("seed", [1, 2])
def test_kmeans_matches_scipy_kmeans2(seed):
    rng = np.random.default_rng(seed)
    x = _clustered(rng, 800, 12, d=16)
    init = x[rng.choice(800, 24, replace=False)].copy()
    init[5] = 50.0                                       # far away: stays empty, keeps its position
    C, codes = oracle.kmeans(x, init, n_iter=6)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        ref_C, ref_codes = scipy_vq.kmeans2(x, init.copy(), iter=6, minit="matrix", missing="warn")
    np.testing.assert_array_equal(codes, ref_codes)
    np.testing.assert_allclose(C, ref_C, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(C[5], init[5])


def test_lloyd_update_brute_force_and_objective_non_increasing():
    rng = np.random.default_rng(3)
    x = rng.integers(-3, 4, (30, 4)).astype(np.float64)
    codes = rng.integers(0, 5, 30)
    codes[codes == 4] = 3                                # centroid 4 has no members
    C = rng.standard_normal((5, 4))
    new = oracle.lloyd_update(x, codes, C)
    for j in range(5):
        rows = [x[i] for i in range(30) if codes[i] == j]
        want = C[j] if not rows else sum(rows) / len(rows)
        np.testing.assert_allclose(new[j], want, rtol=0, atol=1e-14)
    # Lloyd: neither the assignment nor the update step increases the objective
    x = _clustered(rng, 400, 8, d=32)
    C = x[:16].copy()
    prev = np.inf
    for _ in range(5):
        codes = oracle.nn_assign(x, C)
        after_assign = oracle.kmeans_objective(x, codes, C)
        C = oracle.lloyd_update(x, codes, C)
        after_update = oracle.kmeans_objective(x, codes, C)
        assert after_assign <= prev + 1e-12 and after_update <= after_assign + 1e-12
        prev = after_update


def test_qch_equals_ch_when_codebook_holds_every_vector():
    rng = np.random.default_rng(4)
    qo, do = _csr([3, 1, 5]), _csr([2, 4, 1, 6])
    qv, dv = _unit(rng, qo[-1]), _unit(rng, do[-1])
    C = np.vstack([qv, dv])                              # every vector is its own centroid
    qc = np.arange(qo[-1])
    dc = qo[-1] + np.arange(do[-1])
    np.testing.assert_allclose(oracle.qch_dense(qc, qo, dc, do, C), oracle.ch_dense(qv, qo, dv, do), rtol=0,
                               atol=1e-13)
    # and the nearest-centroid map of a vector that is itself a centroid is that centroid
    np.testing.assert_array_equal(oracle.nn_assign(dv, C), dc)


def test_qch_closed_forms_and_empty_sets():
    rng = np.random.default_rng(5)
    C = rng.standard_normal((1, 128))
    qo, do = _csr([4, 0, 2]), _csr([3, 0, 1])
    S = oracle.qch_dense(np.zeros(6, np.int64), qo, np.zeros(4, np.int64), do, C)
    n2 = float(C[0] @ C[0])
    np.testing.assert_allclose(S[0], [4 * n2, -np.inf, 4 * n2])   # one centroid: m_q ||C_0||^2
    np.testing.assert_array_equal(S[1], [0.0, 0.0, 0.0])           # empty query: empty sum
    np.testing.assert_allclose(S[2, [0, 2]], 2 * n2)


def test_qch_invariant_under_relabelling_and_permutation():
    rng = np.random.default_rng(6)
    C = rng.standard_normal((50, 128))
    qc, pc = rng.integers(0, 50, 7), rng.integers(0, 50, 11)
    base = oracle.qch_pair(qc, pc, C)
    perm = rng.permutation(50)                           # centroid j moves to row perm[j]
    C2 = np.empty_like(C)
    C2[perm] = C
    assert oracle.qch_pair(perm[qc], perm[pc], C2) == pytest.approx(base, abs=1e-12)
    assert oracle.qch_pair(rng.permutation(qc), rng.permutation(pc), C) == pytest.approx(base, abs=1e-12)
    # adding a document vector never lowers the score (max over a larger set)
    assert oracle.qch_pair(qc, np.append(pc, 3), C) >= base - 1e-12


def test_qch_within_quantization_error_bound_of_ch():
    rng = np.random.default_rng(7)
    x = _clustered(rng, 2000, 30)
    C, _ = oracle.kmeans(x, x[rng.choice(2000, 64, replace=False)], n_iter=3)
    qo, do = _csr([6, 9, 3]), _csr([5, 12, 8, 1])
    qv, dv = _unit(rng, qo[-1]), x[:do[-1]]
    qc, dc = oracle.nn_assign(qv, C), oracle.nn_assign(dv, C)
    got = oracle.qch_dense(qc, qo, dc, do, C)
    exact = oracle.ch_dense(qv, qo, dv, do)
    # |<NN(q), NN(p)> - <q, p>| <= |NN(q) - q| |NN(p)| + |q| |NN(p) - p|, and a max
    # (then a sum) of terms that each move by at most e moves by at most e (each)
    eq = np.linalg.norm(C[qc] - qv, axis=1)
    ep = np.linalg.norm(C[dc] - dv, axis=1)
    npn = np.linalg.norm(C[dc], axis=1)
    for i in range(3):
        for j in range(4):
            Qi, Pj = slice(qo[i], qo[i + 1]), slice(do[j], do[j + 1])
            e = (eq[Qi][:, None] * npn[Pj][None, :] + ep[Pj][None, :]).max(axis=1).sum()
            assert abs(got[i, j] - exact[i, j]) <= e + 1e-12
    assert np.abs(got - exact).max() > 1e-3                # the estimate is not the exact score


def test_qch_brute_force_loops_and_cands():
    rng = np.random.default_rng(8)
    C = rng.integers(-4, 5, (9, 3)).astype(np.float64)
    qo, do = _csr([2, 3]), _csr([1, 3, 2])
    qc, dc = rng.integers(0, 9, qo[-1]), rng.integers(0, 9, do[-1])
    want = np.zeros((2, 3))
    for i in range(2):
        for j in range(3):
            tot = 0.0
            for a in range(qo[i], qo[i + 1]):
                best = -np.inf
                for b in range(do[j], do[j + 1]):
                    best = max(best, sum(C[qc[a], t] * C[dc[b], t] for t in range(3)))
                tot += best
            want[i, j] = tot
    np.testing.assert_array_equal(oracle.qch_dense(qc, qo, dc, do, C), want)
    co, ids = _csr([3, 2]), np.array([2, 0, 1, 1, 2])
    got = oracle.qch_cands(qc, qo, dc, do, co, ids, C)
    np.testing.assert_array_equal(got, [want[0, 2], want[0, 0], want[0, 1], want[1, 1], want[1, 2]])
