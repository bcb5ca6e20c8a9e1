"""Pins for the oracle's generator and sketches."""
import os

import numpy as np
import pytest
from scipy import stats
from scipy.linalg import hadamard

import workloads as W
from oracle import rng, sketch

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_known_answers():
    want = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    got = [int(rng.draw(0, i)) for i in range(len(want))]
    assert got == want


def test_counter_form_equals_sequential_generator():
    # the counter form must equal stepping the state by GAMMA one output at a time
    key = np.uint64(0x1234567)
    state = int(key)
    for i in range(50):
        state = (state + 0x9E3779B97F4A7C15) & (2 ** 64 - 1)
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & (2 ** 64 - 1)
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & (2 ** 64 - 1)
        z ^= z >> 31
        assert int(rng.draw(key, i)) == z


def test_bucket_range_and_balance():
    h, s = rng.countsketch_draws(42, 200000, 97)
    assert h.min() >= 0 and h.max() < 97
    counts = np.bincount(h[:, 0], minlength=97)
    assert stats.chisquare(counts).pvalue > 1e-4
    assert abs(float(s.astype(float).mean())) < 0.01


def test_sjlt_blocks():
    h, s = rng.countsketch_draws(9, 1000, 12, s=3)
    for b in range(3):
        assert np.all((h[:, b] >= 4 * b) & (h[:, b] < 4 * (b + 1)))
    S = sketch.countsketch_matrix(9, 1000, 12, 3).toarray()
    np.testing.assert_allclose((S * S).sum(0), 1.0)   # each column has unit norm


def test_countsketch_apply_equals_dense_matrix():
    A = W.dense_decay(300, 7, seed=2)
    h, s = rng.countsketch_draws(5, 300, 16)
    S = np.zeros((16, 300))
    S[h[:, 0], np.arange(300)] = s[:, 0]
    np.testing.assert_allclose(sketch.countsketch_apply(A, 5, 16), S @ A, rtol=1e-13, atol=1e-13)


def test_fwht_equals_sylvester_hadamard():
    X = np.random.default_rng(1).standard_normal((64, 3))
    np.testing.assert_allclose(sketch.fwht(X), hadamard(64) @ X, rtol=1e-12, atol=1e-12)


def test_srht_apply_equals_dense_matrix_and_padding():
    A = W.dense_decay(50, 4, seed=3)           # n' = 64, 14 zero rows appended
    S = sketch.srht_matrix(77, 50, 20)
    np.testing.assert_allclose(sketch.srht_apply(A, 77, 20), S @ A, rtol=1e-12, atol=1e-12)


def test_srht_rows_orthogonal():
    # with n = n', S S^T = (n'/m) * [R_k == R_k'] since (H D)(H D)^T = n' I
    S = sketch.srht_matrix(4, 128, 16)
    _, rows, npad = rng.srht_draws(4, 128, 16)
    same = (rows[:, None] == rows[None, :]).astype(float)
    np.testing.assert_allclose(S @ S.T, npad / 16 * same, atol=1e-12)


def test_gaussian_entries_are_standard_normal():
    S = rng.gaussian_matrix(3, 50, 4000)
    z = (S * np.sqrt(50)).reshape(-1)
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1) < 0.01
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # the two values of a Box-Muller pair are independent: uncorrelated, and
    # their squares too
    a, b = z[0::2], z[1::2]
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.01 and abs(np.corrcoef(a * a, b * b)[0, 1]) < 0.01


def test_gaussian_pairs_in_polar_form():
    # pair p in polar form: z_2p^2 + z_2p+1^2 = -2 ln u1 and the angle of
    # (z_2p, z_2p+1) is 2 pi u2, with u1, u2 from draws 2p and 2p + 1; an odd
    # column count puts pairs across rows (entry q = r n + i throughout)
    m, n = 7, 13
    z = rng.gaussian_draws(11, m, n).reshape(-1)
    key = rng.stream_key(11, 3)
    for p in range(0, (m * n) // 2):
        x1 = int(rng.draw(key, 2 * p)) >> 11
        x2 = int(rng.draw(key, 2 * p + 1)) >> 11
        u1 = (x1 + 1) / 2.0 ** 53
        u2 = x2 / 2.0 ** 53
        c, s_ = z[2 * p], z[2 * p + 1]
        assert abs(c * c + s_ * s_ + 2.0 * np.log(u1)) <= 1e-12 * (1.0 - 2.0 * np.log(u1))
        ang = np.arctan2(s_, c) % (2.0 * np.pi)
        d = abs(ang - 2.0 * np.pi * u2)
        assert min(d, 2.0 * np.pi - d) <= 1e-9
    # a row's draws do not depend on m: the first rows of a taller sketch
    np.testing.assert_array_equal(rng.gaussian_draws(11, 9, n)[:m], z.reshape(m, n))


@pytest.mark.parametrize("kind", ["gaussian", "srht", "countsketch"])
def test_sketch_is_unbiased_isometry(kind):
    # E[S^T S] = I: averaged over seeds, ||S a||^2 tracks ||a||^2
    A = W.dense_decay(64, 3, seed=1)
    ratios = []
    for seed in range(200):
        SA = sketch.apply(kind, A, seed, 16)
        ratios.append(np.sum(SA[:, 0] ** 2) / np.sum(A[:, 0] ** 2))
    assert abs(np.mean(ratios) - 1.0) < 0.08


def test_round_bf16_matches_torch_and_ties():
    # torch's CPU float32 -> bfloat16 conversion rounds to nearest, ties to
    # even: an independent implementation of the same rounding
    import torch
    r = np.random.default_rng(3)
    x = np.concatenate([r.standard_normal(20000) * 10.0 ** r.integers(-6, 6, 20000),
                        [0.0, -0.0, 1.0, -2.5]])
    f = x.astype(np.float32)
    ref = torch.from_numpy(f).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(rng.round_bf16(x), ref)
    # exact ties: 1 + 2^-8 sits halfway between 1 and 1 + 2^-7 -> even (1);
    # 1 + 3 * 2^-8 sits between 1 + 2^-7 and 1 + 2^-6 -> even (1 + 2^-6)
    assert rng.round_bf16(1.0 + 2.0 ** -8) == 1.0
    assert rng.round_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


def test_bf16_gaussian_sketch_is_the_rounded_gaussian():
    m, n = 64, 3000
    z = rng.gaussian_draws(5, m, n)
    S = rng.gaussian_matrix(5, m, n)
    S16 = rng.gaussian_matrix_bf16(5, m, n)
    np.testing.assert_allclose(S * np.sqrt(m), z, rtol=1e-15)
    # within half a BF16 unit (2^-8 relative) of the FP64 sketch, and a
    # BF16 value times 1/sqrt(m)
    np.testing.assert_allclose(S16, S, rtol=2.0 ** -8, atol=0)
    q = S16 * np.sqrt(m)
    np.testing.assert_array_equal(rng.round_bf16(q), q)
    # the apply is the product with that matrix
    A = np.random.default_rng(1).standard_normal((n, 4))
    SA = sketch.gaussian_bf16_apply(A, 5, m)
    np.testing.assert_allclose(SA, S16 @ A, rtol=1e-12)


def test_round_e4m3_matches_torch_and_format_facts():
    # torch's float8_e4m3fn conversion rounds to nearest, ties to even (it
    # gives NaN beyond the format's range, so the comparison stays within it)
    import torch
    r = np.random.default_rng(4)
    x = np.concatenate([r.standard_normal(20000) * 2.0 ** r.integers(-12, 9, 20000),
                        [0.0, 1.0, -2.5, 448.0, 464.0, -464.0, 2.0 ** -9, 2.0 ** -10]])
    x = x[np.abs(x) <= 464.0]
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(rng.round_e4m3(x), ref)
    v = rng.e4m3_values()
    assert v[0] == 0.0 and v[1] == 2.0 ** -9 and v[8] == 2.0 ** -6 and v[-1] == 448.0
    assert np.all(np.diff(v) > 0) and v.size == 127
    # ties: 1 + 1/16 between 1 (code even) and 1.125 -> 1; 1 + 3/16 -> 1.25;
    # 2^-10 between 0 and 2^-9 -> 0; 3 * 2^-10 -> 2^-8; saturation beyond 448
    assert rng.round_e4m3(1.0625) == 1.0 and rng.round_e4m3(-1.0625) == -1.0
    assert rng.round_e4m3(1.1875) == 1.25
    assert rng.round_e4m3(2.0 ** -10) == 0.0 and rng.round_e4m3(3 * 2.0 ** -10) == 2.0 ** -8
    assert rng.round_e4m3(470.0) == 448.0 and rng.round_e4m3(-1e6) == -448.0


def test_fp8_terms_scale_and_reconstruction_bound():
    r = np.random.default_rng(8)
    A = r.standard_normal((500, 7)) * np.array([1.0, 1e-3, 1e4, 3.0, 448.0, 0.0, 2.0 ** -20])
    A[0, 1] = 7.0  # one large entry in a small column
    A = A.astype(np.float32).astype(np.float64)
    t, e = sketch.fp8_terms(A)
    mx = np.abs(A).max(axis=0)
    # e_c: the column maximum lands in (224, 448] * 2^e_c; a zero column keeps 0
    nz = mx > 0
    assert np.all(mx[nz] <= np.ldexp(448.0, e[nz])) and np.all(mx[nz] > np.ldexp(224.0, e[nz]))
    assert e[5] == 0 and np.all(t[:, :, 5] == 0)
    # every term is an e4m3 value
    for p in range(3):
        np.testing.assert_array_equal(rng.round_e4m3(t[p]), t[p])
    # three terms leave at most 448 * 2^(e_c - 12) of each entry, and each
    # further term shrinks what is left
    At = sketch.fp8_reconstruct(A)
    assert np.all(np.abs(A - At) <= np.ldexp(448.0, e[None, :] - 12))
    A2 = np.ldexp(t[0] + t[1] / 16.0, e[None, :])
    assert np.abs(A - At).sum() < np.abs(A - A2).sum()
    # exact for values that fit 12 bits in the top binade (and for A = I)
    np.testing.assert_array_equal(sketch.fp8_reconstruct(np.eye(5)), np.eye(5))


def test_fp8_gaussian_sketch_is_the_rounded_gaussian():
    m, n = 64, 3000
    S = rng.gaussian_matrix(5, m, n)
    S8 = rng.gaussian_matrix_fp8(5, m, n)
    # within half an e4m3 unit (2^-4 relative, 2^-10 absolute below 2^-6)
    assert np.all(np.abs(S8 - S) * np.sqrt(m) <= np.maximum(2.0 ** -4 * np.abs(S) * np.sqrt(m),
                                                          2.0 ** -10))
    q = S8 * np.sqrt(m)
    np.testing.assert_array_equal(rng.round_e4m3(q), q)
    A = np.random.default_rng(1).standard_normal((n, 4))
    SA = sketch.gaussian_fp8_apply(A, 5, m)
    np.testing.assert_allclose(SA, S8 @ sketch.fp8_reconstruct(A), rtol=1e-12)
