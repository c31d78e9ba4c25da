"""Pins for the CPU oracle: each test ties it to something other than itself.

Sources of truth used here: the paper's worked example (Sec. 1), closed forms
of Def. 1 for special set shapes, invariants of sum-of-max, reductions of the
problem to single-vector inner-product search (BLAS + sorting), brute-force
rank counting, the OCP FP8 definition, and torch's own float8 / bfloat16 casts.
"""
import math
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import chamfer as och
from oracle import codecs as occ

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _unit(rng, n, d):
    x = rng.standard_normal((n, d))
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def _csr(lengths):
    o = np.zeros(len(lengths) + 1, np.int64)
    o[1:] = np.cumsum(lengths)
    return o


# --------------------------------------------------------------------- CH value
def _read_worked_example():
    vecs, maxes, score = {}, [], None
    with open(os.path.join(GOLDEN, "worked_example_ch.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "max":
                maxes.append((parts[1], float(parts[2]), parts[3]))
            elif parts[0] == "score":
                score = float(parts[1])
            else:
                vecs[parts[0]] = np.array([float(v) for v in parts[1:]])
    Q = np.stack([vecs[f"q{i}"] for i in range(3)])
    P = np.stack([vecs[f"p{i}"] for i in range(4)])
    return Q, P, maxes, score


def test_worked_example_sum_of_row_maxima():
    """Sec. 1: row maxima 0.94, 0.7, 0.22 (p0 reused) sum to 1.86."""
    Q, P, maxes, score = _read_worked_example()
    assert abs(oracle.ch_pair(Q, P) - score) < 1e-12
    # the matched document vector of each query vector is the one the paper names
    for (qn, val, pn) in maxes:
        qi, pi = int(qn[1:]), int(pn[1:])
        assert abs(float(Q[qi] @ P[pi]) - val) < 1e-12
    # the dense and candidate-list forms agree on the same pair
    d = oracle.ch_dense(Q, [0, 3], P, [0, 4])
    assert abs(d[0, 0] - score) < 1e-12
    c = oracle.ch_cands(Q, [0, 3], P, [0, 4], [0, 1], [0])
    assert abs(c[0] - score) < 1e-12
    # distance form (d_X = 1 - <q, p>, Sec. 4.2): sum of minimum distances = m_q - CH
    dist = sum(min(1.0 - float(q @ p) for p in P) for q in Q)
    assert abs(dist - (3 - score)) < 1e-12


def test_closed_form_single_doc_vector():
    """m_p = 1: CH(Q, {p}) = <sum_a a, p> (every a takes the only p)."""
    rng = np.random.default_rng(1)
    for m in (1, 3, 32):
        Q, p = _unit(rng, m, 16), _unit(rng, 1, 16)
        assert abs(oracle.ch_pair(Q, p) - float(Q.sum(axis=0) @ p[0])) < 1e-12


def test_closed_form_single_query_vector_is_mips():
    """m_q = m_p = 1: CH reduces to single-vector inner-product search (BLAS + argsort)."""
    rng = np.random.default_rng(2)
    Q, D = _unit(rng, 5, 32), _unit(rng, 50, 32)
    ones = np.arange(51, dtype=np.int64)
    got = oracle.ch_dense(Q, np.arange(6), D, ones)
    ref = Q @ D.T
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)
    ts, ti = oracle.topk_rows(got, 7)
    np.testing.assert_array_equal(ti, np.argsort(-ref, axis=1, kind="stable")[:, :7])


def test_closed_form_self_similarity_unit_vectors():
    """CH(P, P) = |P| for unit vectors (Cauchy-Schwarz: each p matches itself at 1)."""
    rng = np.random.default_rng(3)
    for m in (1, 7, 64):
        P = _unit(rng, m, 128)
        assert abs(oracle.ch_pair(P, P) - m) < 1e-12


def test_homogeneity():
    """CH(alpha Q, beta P) = alpha beta CH(Q, P) for alpha, beta > 0."""
    rng = np.random.default_rng(4)
    Q, P = rng.standard_normal((5, 8)), rng.standard_normal((9, 8))
    assert abs(oracle.ch_pair(2.0 * Q, 0.25 * P) - 0.5 * oracle.ch_pair(Q, P)) < 1e-12


def test_invariants_permutation_monotone_duplicate_additive():
    rng = np.random.default_rng(5)
    Q, P = _unit(rng, 11, 24), _unit(rng, 17, 24)
    base = oracle.ch_pair(Q, P)
    # permuting document vectors: bitwise equal (each max sees the same values)
    assert oracle.ch_pair(Q, P[rng.permutation(17)]) == base
    # permuting query vectors: equal up to summation order
    assert abs(oracle.ch_pair(Q[rng.permutation(11)], P) - base) < 1e-12
    # adding document vectors never lowers the score
    assert oracle.ch_pair(Q, np.vstack([P, _unit(rng, 3, 24)])) >= base
    # duplicating a document vector changes nothing
    assert oracle.ch_pair(Q, np.vstack([P, P[4:5]])) == base
    # additivity over a partition of the query set
    assert abs(oracle.ch_pair(Q[:4], P) + oracle.ch_pair(Q[4:], P) - base) < 1e-12
    # not symmetric in general: a transposed max would fail the m_p = 1 closed form
    assert abs(oracle.ch_pair(P, Q) - base) > 1e-6


def test_empty_sets():
    """Empty query -> 0 (empty sum); non-empty query vs empty document -> -inf."""
    z = np.zeros((0, 8))
    P = np.ones((2, 8))
    assert oracle.ch_pair(z, P) == 0.0
    assert oracle.ch_pair(P, z) == -math.inf
    d = oracle.ch_dense(np.vstack([P, P]), [0, 0, 2, 4], P, [0, 0, 2])
    assert d[0, 0] == 0.0 and d[0, 1] == 0.0
    assert d[1, 0] == -math.inf and d[1, 1] == pytest.approx(16.0)


def test_dense_and_cands_agree_with_pairwise_on_ragged_sets():
    rng = np.random.default_rng(6)
    ql, dl = [3, 1, 0, 5], [2, 0, 7, 1, 4, 3]
    qv, dv = _unit(rng, sum(ql), 16), _unit(rng, sum(dl), 16)
    qo, do = _csr(ql), _csr(dl)
    dense = oracle.ch_dense(qv, qo, dv, do, max_rows=5)
    for i in range(4):
        for j in range(6):
            ref = oracle.ch_pair(qv[qo[i]:qo[i + 1]], dv[do[j]:do[j + 1]])
            assert dense[i, j] == pytest.approx(ref, abs=1e-12) or (ref == dense[i, j])
    co = np.array([0, 3, 3, 6, 8])
    ci = np.array([5, 1, 2, 0, 0, 4, 3, 2])
    c = oracle.ch_cands(qv, qo, dv, do, co, ci)
    for i in range(4):
        for e in range(co[i], co[i + 1]):
            ref = dense[i, ci[e]]
            assert c[e] == pytest.approx(ref, abs=1e-12) or c[e] == ref


# --------------------------------------------------------------------- top-k
def _rank_count_topk(scores, ids, k):
    """Brute force: an entry's rank is the number of distinct ids that beat it."""
    best = {}
    for s, i in zip(scores, ids):
        if i not in best or s > best[i]:
            best[i] = s
    items = list(best.items())
    ranked = []
    for (i, s) in items:
        r = sum(1 for (j, t) in items if (t > s) or (t == s and j < i))
        ranked.append((r, s, i))
    ranked.sort()
    out_s = [s for (r, s, i) in ranked if r < k]
    out_i = [i for (r, s, i) in ranked if r < k]
    while len(out_s) < k:
        out_s.append(-math.inf)
        out_i.append(-1)
    return np.array(out_s), np.array(out_i)


@pytest.mark.parametrize("seed", range(8))
def test_topk_matches_rank_counting(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 40))
    scores = rng.choice([0.5, 1.0, -2.0, 3.0], size=n) if seed % 2 else rng.standard_normal(n)
    ids = rng.integers(0, 30, size=n)           # repeated ids on purpose
    for k in (1, 5, 64):
        ts, ti = och._topk_one(np.asarray(scores, float), ids, k)
        rs, ri = _rank_count_topk(list(scores), list(ids), k)
        np.testing.assert_array_equal(ti, ri)
        np.testing.assert_array_equal(ts, rs)


def test_topk_segments_positions_and_padding():
    s = np.array([0.1, 0.9, 0.9, -1.0, 5.0])
    ts, ti = oracle.topk_segments(s, [0, 4, 4, 5], 3)
    np.testing.assert_array_equal(ti[0], [1, 2, 0])     # tie 0.9 -> smaller position first
    np.testing.assert_array_equal(ti[1], [-1, -1, -1])  # empty segment -> padding
    np.testing.assert_array_equal(ti[2], [0, -1, -1])
    assert ts[1, 0] == -math.inf


def test_padding_ids_never_ranked():
    """A negative id is padding: even with the best score it enters neither a
    top-k nor the beam, and the rest rank as if it were absent."""
    ts, ti = oracle.topk_segments(np.array([9.0, 1.0, 9.0, 2.0]), [0, 4], 3, seg_ids=np.array([-1, 4, -7, 3]))
    np.testing.assert_array_equal(ti[0], [3, 4, -1])
    np.testing.assert_array_equal(ts[0], [2.0, 1.0, -math.inf])
    bs, bi = oracle.beam_merge(np.array([[5.0, -math.inf]]), np.array([[8, -1]]), np.array([7.0, 6.0, 4.0]),
                               [0, 3], np.array([-1, 2, -1]), 2)
    np.testing.assert_array_equal(bi[0], [2, 8])
    np.testing.assert_array_equal(bs[0], [6.0, 5.0])


# --------------------------------------------------------------------- beam (bounded R)
def test_beam_replay_equals_one_shot_top_ef():
    """After any number of steps the bounded beam equals the top-ef of everything
    inserted so far (Alg. 5 keeps at most ef, evicting the worst)."""
    rng = np.random.default_rng(7)
    n_q, ef = 3, 10
    steps, all_s, all_i = [], [[] for _ in range(n_q)], [[] for _ in range(n_q)]
    for st in range(6):
        lens = rng.integers(0, 9, size=n_q)
        co = _csr(lens)
        ci = rng.integers(0, 40, size=co[-1])
        # a document keeps one score across steps, as a deterministic estimate would
        cs = np.sin(ci * 1.7 + np.repeat(np.arange(n_q), lens))
        steps.append((cs, co, ci))
        for q in range(n_q):
            all_s[q] += list(cs[co[q]:co[q + 1]])
            all_i[q] += list(ci[co[q]:co[q + 1]])
    bs, bi = oracle.beam_replay(n_q, ef, steps)
    for q in range(n_q):
        rs, ri = _rank_count_topk(all_s[q], all_i[q], ef)
        np.testing.assert_array_equal(bi[q], ri)
        np.testing.assert_array_equal(bs[q], rs)


# --------------------------------------------------------------------- recall
def test_recall_definitions():
    ex = np.array([5.0, 4.0, 3.0, 3.0, 1.0])
    assert oracle.recall_at_k([0, 1, 2], ex, 3) == 1.0
    assert oracle.recall_at_k([0, 1, 3], ex, 3) == 1.0      # tie at the 3rd place
    assert oracle.recall_at_k([0, 1, 4], ex, 3) == pytest.approx(2 / 3)
    assert oracle.recall_at_k([4, 4, 4], ex, 3) == 0.0
    ok, bad, missing = oracle.tie_aware_match([0, 1, 3], ex, 3, 0.0)
    assert ok
    ok, bad, missing = oracle.tie_aware_match([0, 2, 4], ex, 3, 0.0)
    assert not ok and bad == 1 and missing == 1


# --------------------------------------------------------------------- codecs
def test_e4m3_decode_table_from_ocp_definition():
    t = oracle.e4m3_decode_table()
    assert t[0x7E] == 448.0 and t[0xFE] == -448.0           # largest finite
    assert t[0x08] == 2.0 ** -6                            # smallest normal
    assert t[0x01] == 2.0 ** -9                            # smallest subnormal
    assert t[0x38] == 1.0 and t[0x00] == 0.0
    assert math.isnan(t[0x7F]) and math.isnan(t[0xFF])
    assert np.signbit(t[0x80])
    assert np.count_nonzero(np.isnan(t)) == 2              # no infinities, two NaNs
    # torch's independent float8_e4m3fn implementation
    ref = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    same = (t == ref) | (np.isnan(t) & np.isnan(ref))
    assert same.all()


def test_e4m3_encode_matches_torch_on_all_midpoints_and_sweep():
    t = oracle.e4m3_decode_table()[:0x7F]
    mids = (t[1:] + t[:-1]) / 2
    x = np.concatenate([t, mids, np.nextafter(mids, 0), np.nextafter(mids, 1e9)])
    rng = np.random.default_rng(8)
    x = np.concatenate([x, rng.uniform(-448, 448, 200000), rng.uniform(-1, 1, 200000) * 2.0 ** -6])
    x = np.concatenate([x, -x]).astype(np.float32)
    got = oracle.e4m3_encode(x.astype(np.float64))
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    np.testing.assert_array_equal(got, ref)
    # saturation (torch does not saturate, so check against the definition)
    big = oracle.e4m3_encode(np.array([448.0, 460.0, 1e6, -1e6]))
    np.testing.assert_array_equal(big, [0x7E, 0x7E, 0x7E, 0xFE])
    assert oracle.e4m3_encode(np.array([np.nan]))[0] == 0x7F


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(9)
    x = rng.standard_normal(300000).astype(np.float32) * np.float32(10.0) ** rng.integers(-30, 30, 300000).astype(np.float32)
    # exact halfway cases: low 16 bits = 0x8000, both parities
    expo = rng.integers(1, 254, 1000, dtype=np.uint32) << 23
    man = rng.integers(0, 2 ** 7, 1000, dtype=np.uint32) << 16
    sign = rng.integers(0, 2, 1000, dtype=np.uint32) << 31
    hb = sign | expo | man | np.uint32(0x8000)          # dropped half is exactly 0x8000
    hb2 = hb ^ np.uint32(0x10000)                       # the other parity of the kept LSB
    x = np.concatenate([x, hb.view(np.float32), hb2.view(np.float32), np.array([0.0, -0.0, 3.4e38], np.float32)])
    got = oracle.bf16_round_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(got, ref)
    np.testing.assert_array_equal(oracle.bf16_decode(got), torch.from_numpy(x).to(torch.bfloat16).double().numpy())


def test_pow2_scale_is_minimal_power_of_two():
    rng = np.random.default_rng(10)
    vals = np.concatenate([rng.uniform(0, 1, 2000), [448.0, 224.0, 1.0, 2.0 ** -20, 1e30]])
    for a in vals.astype(np.float32):
        s = oracle.pow2_scale(float(a))
        m, e = math.frexp(s)
        assert m == 0.5                                   # power of two
        if a == 0:
            assert s == 1.0
            continue
        assert a <= 448.0 * s
        assert a > 448.0 * s / 2                          # half of it would not do
    assert oracle.pow2_scale(0.0) == 1.0
    assert oracle.pow2_scale(1e-45) == 2.0 ** -126        # clamp keeps a normal float32


def test_quantize_fp8_roundtrip_bound():
    rng = np.random.default_rng(11)
    x = _unit(rng, 500, 128).astype(np.float32)
    codes, scales = oracle.quantize_fp8(x)
    assert codes.dtype == np.uint8 and scales.dtype == np.float32
    deq = oracle.dequantize_fp8(codes, scales)
    ratio = np.abs(x.astype(np.float64)) / scales[:, None]
    assert ratio.max() <= 448.0
    # relative rounding error of E4M3 (3 mantissa bits) in the normal range is <= 2^-4
    normal = ratio >= 2.0 ** -6
    rel = np.abs(deq - x)[normal] / np.abs(x)[normal]
    assert rel.max() <= 2.0 ** -4 + 1e-12
    # subnormal range: absolute error <= half the subnormal spacing
    sub = ~normal
    assert (np.abs(deq - x)[sub] / np.broadcast_to(scales[:, None], x.shape)[sub]).max() <= 2.0 ** -10 + 1e-15


# --- the split of float32 values into two bfloat16 parts (exact mode on
# three bfloat16 products)

def _bf16_values(rng, n):
    """Random finite bfloat16 values (as float64) over a wide exponent range."""
    expo = rng.integers(60, 190, n, dtype=np.uint32) << 23
    man = rng.integers(0, 2 ** 7, n, dtype=np.uint32) << 16
    sign = rng.integers(0, 2, n, dtype=np.uint32) << 31
    return (sign | expo | man).view(np.float32).astype(np.float64)


def test_split_bf16x3_round_trips_exact_two_part_values():
    # x = h + l with bfloat16 h and l, |l| at most a quarter of h's bfloat16
    # ulp: such an x is a float32 whose nearest bfloat16 is h, and x - h = l
    # is itself a bfloat16, so the split must return exactly (h, l)
    rng = np.random.default_rng(21)
    h = _bf16_values(rng, 20000)
    ulp = np.ldexp(1.0, np.frexp(np.abs(h))[1] - 8)            # bfloat16 spacing at |h|
    frac = rng.integers(-2 ** 6, 2 ** 6 + 1, h.size) / 2.0 ** 8  # |l| <= ulp / 4, on an 8-bit grid
    l = frac * ulp
    x = (h + l).astype(np.float32)
    assert (x.astype(np.float64) == h + l).all()                 # representable exactly
    hi, lo = oracle.split_bf16x3(x)
    np.testing.assert_array_equal(oracle.bf16_decode(hi), h)
    np.testing.assert_array_equal(oracle.bf16_decode(lo), l)
    # a bfloat16 value splits into itself and zero
    hi, lo = oracle.split_bf16x3(h.astype(np.float32))
    np.testing.assert_array_equal(oracle.bf16_decode(hi), h)
    assert (oracle.bf16_decode(lo) == 0.0).all()


def test_split_bf16x3_parts_match_torch_and_the_error_bound():
    rng = np.random.default_rng(22)
    x = (rng.standard_normal(200000) * 10.0 ** rng.integers(-20, 20, 200000)).astype(np.float32)
    hi, lo = oracle.split_bf16x3(x)
    t = torch.from_numpy(x)
    th = t.to(torch.bfloat16)
    rest = t - th.to(torch.float32)                               # exact in float32
    np.testing.assert_array_equal(hi, th.view(torch.int16).numpy().view(np.uint16))
    np.testing.assert_array_equal(lo, rest.to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16))
    err = np.abs(x.astype(np.float64) - oracle.bf16_decode(hi) - oracle.bf16_decode(lo))
    assert (err <= 2.0 ** -16 * np.abs(x.astype(np.float64))).all()


def test_ch_bf16x3_reduces_to_ch_on_bfloat16_values_and_stays_within_the_product_bound():
    rng = np.random.default_rng(23)
    q_off = np.array([0, 3, 7, 7, 12])
    d_off = np.array([0, 5, 6, 6, 14, 20])
    Q = rng.standard_normal((12, 128)).astype(np.float32)
    D = rng.standard_normal((20, 128)).astype(np.float32)
    # bfloat16-valued inputs: every lo part is zero and the three-product form
    # is the exact inner product
    Qb = oracle.bf16_decode(oracle.bf16_round_bits(Q)).astype(np.float32)
    Db = oracle.bf16_decode(oracle.bf16_round_bits(D)).astype(np.float32)
    np.testing.assert_array_equal(oracle.ch_dense_bf16x3(Qb, q_off, Db, d_off), oracle.ch_dense(Qb, q_off, Db, d_off))
    # general inputs: with a = ah + al + ea, |al| <= (1 + 2^-8) 2^-8 |a| and
    # |ea| <= 2^-16 |a| (likewise p), the dropped terms ah*ep + al*pl + ea*ph
    # + al*ep + ea*pl + ea*ep of a*p add up to at most 3.1 * 2^-16 |a||p|, and
    # a max moves by at most the largest change of its arguments
    got = oracle.ch_dense_bf16x3(Q, q_off, D, d_off)
    ref = oracle.ch_dense(Q, q_off, D, d_off)
    absQ, absD = np.abs(Q.astype(np.float64)), np.abs(D.astype(np.float64))
    bound = np.zeros_like(ref)
    for i in range(len(q_off) - 1):
        for j in range(len(d_off) - 1):
            if q_off[i] == q_off[i + 1]:
                continue
            if d_off[j] == d_off[j + 1]:
                continue
            B = absQ[q_off[i]:q_off[i + 1]] @ absD[d_off[j]:d_off[j + 1]].T
            bound[i, j] = 3.1 * 2.0 ** -16 * B.max(axis=1).sum()
    fin = np.isfinite(ref)
    assert (np.abs(got[fin] - ref[fin]) <= bound[fin]).all()
    np.testing.assert_array_equal(np.isfinite(got), fin)
    # the difference is real (the mode is not the float32 products) and small
    assert np.abs(got[fin] - ref[fin]).max() > 0
    # candidate lists give the same values as the dense matrix
    c_off = np.array([0, 2, 2, 5, 6])
    c_ids = np.array([4, 0, 1, 3, 0, 2])
    cand = oracle.ch_cands_bf16x3(Q, q_off, D, d_off, c_off, c_ids)
    want = np.concatenate([got[i, c_ids[c_off[i]:c_off[i + 1]]] for i in range(4)])
    np.testing.assert_array_equal(cand, want)
