"""GPU parity of every step of the HIP path against the FP64 oracle.

Step-level calls (draws, sketch, factor, A^T A products) are compared with the
oracle's independent implementations; the whole path is compared with the
direct per-lambda solve at 1e-6 relative error per lambda.
"""
import numpy as np
import pytest

import workloads as W
from oracle import direct, ihs_bin, rng, sketch

pytestmark = pytest.mark.gpu

TOL_PATH = 1e-6


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    from paper_2210_12212_amd import Context
    c = Context(0)
    yield c
    c.close()


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def csr_dev(torch, M):
    from paper_2210_12212_amd import CsrInput
    return CsrInput(dev(torch, M.row_ptr), dev(torch, M.col_idx), dev(torch, M.vals), M.n, M.d)


# ---------------------------------------------------------------- products
@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("n,d,w", [(300, 70, 5), (257, 33, 40), (1000, 130, 100), (64, 64, 1),
                                   (2048, 100, 7), (3001, 257, 33), (4099, 64, 130),
                                   (1500, 90, 200), (2000, 1100, 20), (1300, 1030, 65)])
def test_ata_dense(torch, ctx, dt, n, d, w):
    r = np.random.default_rng(n + d + w)
    A = r.standard_normal((n, d)).astype(dt)
    U = r.standard_normal((d, w))
    Wg = ctx.ata_apply(dev(torch, A), dev(torch, U)).cpu().numpy()
    A64 = A.astype(np.float64)
    ref = A64.T @ (A64 @ U)
    np.testing.assert_allclose(Wg, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("w,ldu", [(23, 32), (69, 128), (138, 192), (253, 256)])
def test_ata_ragged_width_ignores_padding(torch, ctx, w, ldu):
    # columns [w, ldu) of U are read by whole column tiles but must not matter:
    # they hold NaN here, and only columns [0, w) of W are written
    r = np.random.default_rng(w)
    A = r.standard_normal((3000, 200)).astype(np.float32)
    Ufull = r.standard_normal((200, ldu))
    Ufull[:, w:] = np.nan
    Ut = dev(torch, Ufull)[:, :w]
    assert Ut.stride(0) == ldu
    Wg = ctx.ata_apply(dev(torch, A), Ut).cpu().numpy()
    A64 = A.astype(np.float64)
    ref = A64.T @ (A64 @ Ufull[:, :w])
    assert np.isfinite(Wg).all()
    np.testing.assert_allclose(Wg, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("n,d,per,w", [(20000, 500, 9, 3), (5000, 64, 20, 70), (3000, 1000, 2, 1),
                                       (1, 7, 3, 5)])
def test_ata_csr_skewed_columns(torch, ctx, n, d, per, w):
    # column 0 holds nearly every row (many gather chunks); w from 1 to 70
    M = W.csr_zipf(n, d, per, seed=n + w, dtype=np.float64)
    U = np.random.default_rng(w).standard_normal((d, w))
    Wg = ctx.ata_apply(csr_dev(torch, M), dev(torch, U)).cpu().numpy()
    ref = ihs_bin.Operator(M).AtA(U)
    np.testing.assert_allclose(Wg, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())
    # the gather sums in a fixed order: the same bits again
    W2 = ctx.ata_apply(csr_dev(torch, M), dev(torch, U)).cpu().numpy()
    np.testing.assert_array_equal(Wg, W2)


def test_ata_csr(torch, ctx):
    M = W.csr_zipf(2000, 300, 7, seed=3, dtype=np.float32)
    U = np.random.default_rng(1).standard_normal((300, 9))
    Wg = ctx.ata_apply(csr_dev(torch, M), dev(torch, U)).cpu().numpy()
    op = ihs_bin.Operator(M)
    ref = op.AtA(U)
    np.testing.assert_allclose(Wg, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


# ---------------------------------------------------------------- sketches
@pytest.mark.parametrize("n,m,s", [(1000, 37, 1), (4099, 64, 4), (1, 5, 1)])
def test_countsketch_draws_bit_exact(torch, ctx, n, m, s):
    kind = "sjlt" if s > 1 else "countsketch"
    idx, sign = ctx.sketch_draws(kind, 12345, n, m, s)
    h, sg = rng.countsketch_draws(12345, n, m, s)
    assert np.array_equal(idx.cpu().numpy(), h)
    assert np.array_equal(sign.cpu().numpy(), sg)


@pytest.mark.parametrize("n,m", [(1000, 100), (4096, 333), (3, 7)])
def test_srht_draws_bit_exact(torch, ctx, n, m):
    rows, sign = ctx.sketch_draws("srht", 99, n, m)
    sg, rr, _ = rng.srht_draws(99, n, m)
    assert np.array_equal(sign.cpu().numpy(), sg)
    assert np.array_equal(rows.cpu().numpy(), rr)


@pytest.mark.parametrize("kind", ["countsketch", "srht", "gaussian", "sjlt"])
@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_sketch_apply_dense(torch, ctx, kind, dt):
    A = W.dense_decay(1500, 45, seed=4, dtype=dt)   # n' = 2048 for SRHT (zero padding)
    m = 96
    SA = ctx.sketch_apply(dev(torch, A), kind, m, 321, sjlt_s=4).cpu().numpy()
    ref = sketch.apply(kind, A, 321, m, s=4)
    # the Gaussian entries go through device log/cos/sqrt: allow a few ulp
    tol = 1e-12 if kind != "gaussian" else 1e-11
    np.testing.assert_allclose(SA, ref, rtol=tol, atol=tol * np.abs(ref).max())


@pytest.mark.parametrize("kind", ["countsketch", "srht"])
def test_sketch_apply_csr(torch, ctx, kind):
    M = W.csr_zipf(3000, 120, 5, seed=9, dtype=np.float32)
    SA = ctx.sketch_apply(csr_dev(torch, M), kind, 64, 77).cpu().numpy()
    ref = sketch.apply(kind, M, 77, 64)
    np.testing.assert_allclose(SA, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_srht_large_order_three_passes(torch, ctx):
    # n' = 2^19 needs three Walsh-Hadamard passes over row digits
    A = W.dense_decay((1 << 18) + 5, 3, seed=5, dtype=np.float32)
    SA = ctx.sketch_apply(dev(torch, A), "srht", 50, 8).cpu().numpy()
    ref = sketch.apply("srht", A, 8, 50)
    np.testing.assert_allclose(SA, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


# ---------------------------------------------------------------- factor
@pytest.mark.parametrize("d", [40, 64, 200, 300, 1000, 2100])
def test_precond_factor(torch, ctx, d):
    r = np.random.default_rng(d)
    SA = r.standard_normal((d // 2 + 3, d))
    lam0 = np.array([1e-3, 0.5, 7.0])
    Lf, Li = ctx.precond_factor(dev(torch, SA), lam0)
    Lf, Li = Lf.cpu().numpy(), Li.cpu().numpy()
    for t, l0 in enumerate(lam0):
        H = SA.T @ SA + l0 * np.eye(d)
        assert np.allclose(np.triu(Lf[t], 1), 0)
        np.testing.assert_allclose(Lf[t] @ Lf[t].T, H, rtol=1e-11, atol=1e-11 * np.abs(H).max())
        Lref = np.linalg.cholesky(H)
        np.testing.assert_allclose(Lf[t], Lref, rtol=1e-8, atol=1e-9 * np.abs(Lref).max())
        np.testing.assert_allclose(Li[t] @ Lf[t], np.eye(d), atol=1e-8)


def test_precond_not_spd_is_reported(torch, ctx):
    from paper_2210_12212_amd import IhsbinError
    SA = np.zeros((4, 8))
    with pytest.raises(IhsbinError):
        ctx.precond_factor(dev(torch, SA), [-1.0])


# ---------------------------------------------------------------- basis
@pytest.mark.parametrize("centred", [1, 0])
def test_basis_matches_oracle_recursion(torch, ctx, centred):
    # same sketch, same step sizes, same k: the GPU basis equals the oracle's
    A = W.dense_decay(800, 40, seed=12)
    B, _ = W.rhs(A, 2, 0.1, seed=13)
    lo, hi, k = 1e-2, 1e1, 6
    grid, lam0 = ihs_bin.plan(lo, hi)
    taus = [0.9 - 0.01 * l for l in range(len(lam0))]
    path, rep = ctx.path_build(dev(torch, A), dev(torch, B), lo, hi, sketch="countsketch", m=160,
                               seed=55, adaptive_m=0, k_fixed=k, taus=taus, centred=centred)
    SA = sketch.apply("countsketch", A, 55, 160)
    op = ihs_bin.Operator(A)
    C = op.At(B)
    iv = path.intervals()
    np.testing.assert_allclose(iv["lo"], grid[:-1], rtol=1e-14)
    np.testing.assert_allclose(iv["lam0"], lam0, rtol=1e-14)
    assert list(iv["k"]) == [k] * len(lam0)
    for l in (0, len(lam0) // 2, len(lam0) - 1):
        P = ihs_bin.Precond(SA, lam0[l])
        ref_pt = lam0[l] if centred else 0.0
        ut = ihs_bin.basis(op, P, C, taus[l], k, ref_pt)
        got = path.basis(l).cpu().numpy()
        for j in range(k):
            scale = np.abs(ut[j]).max()
            np.testing.assert_allclose(got[j], ut[j], rtol=1e-8, atol=1e-9 * scale)
    lams = W.lambda_grid(lo, hi, 11)
    Xo, _ = ihs_bin.path(A, B, lams, SA, lo, hi, k=k, taus=taus, centred=bool(centred))
    X = path.eval(lams).cpu().numpy()
    assert direct.rel_err(X, Xo).max() < 1e-9
    path.free()


# ---------------------------------------------------------------- path
def _check_path(X, A, B, lams, tol=TOL_PATH):
    ref = direct.ridge_path(A, B, lams)
    err = direct.rel_err(X, ref)
    assert err.max() <= tol, f"max rel err {err.max():.3e} at lambda {lams[int(err.argmax())]:.3e}"
    return err


def test_path_dense_decay_2048x256(torch, ctx):
    p = W.make("dense_decay_2048x256")
    path, rep = ctx.path_build(dev(torch, p.A), dev(torch, p.B), p.lam_min, p.lam_max,
                               sketch=p.sketch, m=p.m, seed=p.sketch_seed)
    assert rep["status"] == 0, rep
    X = path.eval(p.lambdas).cpu().numpy()
    err = _check_path(X, p.A, p.B, p.lambdas)
    print(f"dense_decay: m_used={rep['m_used']} k_max={rep['k_max_used']} max_err={err.max():.2e}")
    path.free()


@pytest.mark.parametrize("kind", ["gaussian", "srht", "countsketch", "sjlt"])
def test_path_each_sketch_matrix_rhs(torch, ctx, kind):
    A = W.dense_decay(1200, 60, seed=21, dtype=np.float32)
    B, _ = W.rhs(A, 3, 0.1, seed=22)
    lams = W.lambda_grid(1e-3, 1e2, 23)
    X, rep = ctx.solve_path(dev(torch, A), dev(torch, B), lams, sketch=kind, m=120, seed=4, sjlt_s=2)
    assert rep["status"] == 0, rep
    _check_path(X.cpu().numpy(), A, B, lams)


@pytest.mark.parametrize("prec,fmt", [("f64", "dense"), ("bf16", "dense"), ("fp8", "dense"),
                                      ("f64", "csr")])
def test_gaussian_growth_keeps_rows(torch, ctx, prec, fmt):
    # a Gaussian sketch grown by the probes keeps the rows it has formed
    # (rescaled); the path must equal, up to rounding, the one built with the
    # final m drawn at once, and both must match the oracle
    if fmt == "csr":
        A = W.csr_zipf(6000, 150, 10, seed=41, dtype=np.float32)
        Ad = csr_dev(torch, A)
    else:
        A = W.dense_decay(6000, 150, seed=41, dtype=np.float32)
        Ad = dev(torch, A)
    B, _ = W.rhs(A, 2, 0.1, seed=42)
    lams = W.lambda_grid(1e-3, 1e2, 21)
    sp = {"f64": 0, "bf16": 1, "fp8": 2}[prec]
    X1, r1 = ctx.solve_path(Ad, dev(torch, B), lams, sketch="gaussian", m=16, seed=5,
                            adaptive_m=1, sketch_prec=sp, rate_target=0.3)
    assert r1["status"] == 0 and r1["sketch_trials"] >= 2, r1
    X2, r2 = ctx.solve_path(Ad, dev(torch, B), lams, sketch="gaussian", m=r1["m_used"], seed=5,
                            adaptive_m=0, sketch_prec=sp, rate_target=0.3)
    assert r2["status"] == 0 and r2["m_used"] == r1["m_used"], (r1, r2)
    X1, X2 = X1.cpu().numpy(), X2.cpu().numpy()
    assert direct.rel_err(X1, X2).max() <= 1e-9
    _check_path(X1, A, B, lams)


@pytest.mark.parametrize("prec", [0, 1])
def test_gaussian_exact_switch(torch, ctx, prec):
    # adaptive_m = 3: a Gaussian sketch that would need more rows than the
    # exact Gram costs (d for FP64, 8 d for BF16) is replaced by S = I (m = n);
    # a sketch that meets the target first is kept as the spectral policy has it
    A = W.dense_decay(6000, 150, seed=61, dtype=np.float32)
    B, _ = W.rhs(A, 2, 0.1, seed=62)
    lams = W.lambda_grid(1e-3, 1e2, 21)
    Ad, Bd = dev(torch, A), dev(torch, B)
    X, rep = ctx.solve_path(Ad, Bd, lams, sketch="gaussian", m=64, seed=5, adaptive_m=3,
                            sketch_prec=prec, rate_target=0.05)
    assert rep["status"] == 0 and rep["m_used"] == 6000, rep
    _check_path(X.cpu().numpy(), A, B, lams)
    if prec == 0:
        return  # an FP64 Gaussian sketch of d rows already costs the exact Gram
    X1, r1 = ctx.solve_path(Ad, Bd, lams, sketch="gaussian", m=300, seed=5, adaptive_m=1,
                            sketch_prec=prec, rate_target=0.9)
    X3, r3 = ctx.solve_path(Ad, Bd, lams, sketch="gaussian", m=300, seed=5, adaptive_m=3,
                            sketch_prec=prec, rate_target=0.9)
    assert r3["m_used"] == r1["m_used"] <= 8 * 150, (r1, r3)
    assert np.array_equal(X1.cpu().numpy(), X3.cpu().numpy())


def test_gaussian_exact_switch_leaves_csr_sketched(torch, ctx):
    # S = I would copy a CSR matrix densely: for CSR A the policy stays the
    # spectral one (same m and path as adaptive_m = 1)
    M = W.csr_zipf(6000, 150, 10, seed=63, dtype=np.float32)
    B, _ = W.rhs(M, 1, 0.1, seed=64)
    lams = W.lambda_grid(1e-3, 1e2, 15)
    Md, Bd = csr_dev(torch, M), dev(torch, B)
    X1, r1 = ctx.solve_path(Md, Bd, lams, sketch="gaussian", m=64, seed=5, adaptive_m=1,
                            rate_target=0.05)
    X3, r3 = ctx.solve_path(Md, Bd, lams, sketch="gaussian", m=64, seed=5, adaptive_m=3,
                            rate_target=0.05)
    assert r3["m_used"] == r1["m_used"], (r1, r3)
    assert np.array_equal(X1.cpu().numpy(), X3.cpu().numpy())
    _check_path(X3.cpu().numpy(), M, B, lams)


def test_path_csr(torch, ctx):
    M = W.csr_zipf(6000, 200, 8, seed=31, dtype=np.float32)
    B, _ = W.rhs(M, 1, 0.1, seed=32)
    lams = W.lambda_grid(1e-2, 1e2, 17)
    X, rep = ctx.solve_path(csr_dev(torch, M), dev(torch, B), lams, sketch="countsketch", m=400, seed=3)
    assert rep["status"] == 0, rep
    _check_path(X.cpu().numpy(), M, B, lams)


def test_eval_any_order_and_float32_output(torch, ctx):
    A = W.dense_decay(900, 30, seed=41)
    B, _ = W.rhs(A, 1, 0.1, seed=42)
    path, _ = ctx.path_build(dev(torch, A), dev(torch, B), 1e-2, 1e1, sketch="srht", m=64, seed=1)
    lams = np.array([3.0, 1e-2, 1e1, 0.05, 0.05])
    X64 = path.eval(lams).cpu().numpy()
    X32 = path.eval(lams, dtype=torch.float32).cpu().numpy()
    _check_path(X64, A, B, lams)
    np.testing.assert_allclose(X32, X64, rtol=1e-6, atol=1e-7 * np.abs(X64).max())
    np.testing.assert_array_equal(X64[3], X64[4])
    path.free()


def test_errors(torch, ctx):
    from paper_2210_12212_amd import IhsbinError
    A = W.dense_decay(100, 10, seed=1)
    B, _ = W.rhs(A, 1, 0.1, seed=2)
    path, _ = ctx.path_build(dev(torch, A), dev(torch, B), 0.1, 1.0, sketch="gaussian", m=20)
    with pytest.raises(IhsbinError) as e:
        path.eval([2.0])
    assert e.value.status == -6
    path.free()
    with pytest.raises(IhsbinError) as e:
        ctx.path_build(dev(torch, A), dev(torch, B), 1.0, 0.1)
    assert e.value.status == -1
    At = np.ascontiguousarray(A[:8])  # n < d: built on the dual problem
    path, _ = ctx.path_build(dev(torch, At), dev(torch, B[:8]), 0.1, 1.0)
    assert path.dual == 1 and path.d == 10
    path.free()
    bad = W.csr_zipf(50, 10, 3, seed=1)
    bad.col_idx[5] = 10
    with pytest.raises(IhsbinError) as e:
        ctx.ata_apply(csr_dev(torch, bad), dev(torch, np.ones((10, 1))))
    assert e.value.status == -1


def test_k_max_reached_reports_noconv(torch, ctx):
    A = W.dense_decay(600, 40, seed=51)
    B, _ = W.rhs(A, 1, 0.1, seed=52)
    path, rep = ctx.path_build(dev(torch, A), dev(torch, B), 1e-3, 1e2, sketch="gaussian", m=80,
                               adaptive_m=0, k_max=2)
    assert rep["status"] == -5 and rep["n_unconverged"] > 0
    X = path.eval([1e-3, 1.0]).cpu().numpy()   # still usable
    assert np.all(np.isfinite(X))
    path.free()


@pytest.mark.parametrize("kind,fmt", [("srht", "dense"), ("countsketch", "dense"),
                                      ("sjlt", "dense"), ("gaussian", "dense"),
                                      ("countsketch", "csr"), ("sjlt", "csr"), ("gaussian", "csr")])
def test_run_twice_identical(torch, ctx, kind, fmt):
    # every sum runs in a fixed order (sketches, products, reductions): the
    # same inputs give the same bits
    if fmt == "dense":
        A = W.dense_decay(3000, 50, seed=61)
        Ad = dev(torch, A)
    else:
        A = W.csr_zipf(6000, 90, 7, seed=61, dtype=np.float32)
        Ad = csr_dev(torch, A)
    B, _ = W.rhs(A, 2, 0.1, seed=62)
    lams = W.lambda_grid(1e-3, 1e2, 9)
    X1, _ = ctx.solve_path(Ad, dev(torch, B), lams, sketch=kind, m=100, seed=5, sjlt_s=2)
    X2, _ = ctx.solve_path(Ad, dev(torch, B), lams, sketch=kind, m=100, seed=5, sjlt_s=2)
    assert torch.equal(X1, X2)
    SA1 = ctx.sketch_apply(Ad, kind, 64, 9, sjlt_s=2)
    SA2 = ctx.sketch_apply(Ad, kind, 64, 9, sjlt_s=2)
    assert torch.equal(SA1, SA2)


def test_step_sizes_close_to_exact_spectrum(torch, ctx):
    # the Lanczos estimates at the interval ends give tau close to the exact
    # minimax step over the interval (slightly smaller: the largest eigenvalue
    # is raised by its residual bound)
    A = W.dense_decay(900, 48, seed=71)
    B, _ = W.rhs(A, 1, 0.1, seed=72)
    lo, hi = 1e-2, 1e1
    path, rep = ctx.path_build(dev(torch, A), dev(torch, B), lo, hi, sketch="countsketch", m=200,
                               seed=9, adaptive_m=0, lanczos_steps=40)
    iv = path.intervals()
    SA = sketch.apply("countsketch", A, 9, 200)
    op = ihs_bin.Operator(A)
    for l in range(len(iv["lam0"])):
        P = ihs_bin.Precond(SA, iv["lam0"][l])
        tau_exact, rate_exact = ihs_bin.step_size_from_bounds(
            *ihs_bin.interval_bounds(op, P, iv["lo"][l], iv["hi"][l]))
        assert 0.9 * tau_exact <= iv["tau"][l] <= 1.0 * tau_exact, (l, iv["tau"][l], tau_exact)
        assert iv["rate"][l] >= rate_exact - 1e-9
    path.free()


# ---------------------------------------------------------------- dual (n < d)
@pytest.mark.parametrize("kind", ["gaussian", "srht", "countsketch"])
@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_dual_path_matches_direct(torch, ctx, kind, dt):
    # Section 5.2: n < d is built on (A A^T + lam I) z = b, x = A^T z
    A = W.dense_decay(300, 1200, seed=81, dtype=dt)
    B, _ = W.rhs(A, 2, 0.1, seed=82)
    lams = W.lambda_grid(1e-2, 1e3, 15)
    path, rep = ctx.path_build(dev(torch, A), dev(torch, B), 1e-2, 1e3, sketch=kind, m=150,
                               seed=83, tol=1e-9)
    assert path.dual == 1 and path.d == 1200 and rep["n_unconverged"] == 0, rep
    X = path.eval(lams).cpu().numpy()
    path.free()
    ref = direct.ridge_path_dual(A, B, lams)
    err = direct.rel_err(X, ref)
    assert err.max() <= 1e-6, err


def test_dual_csr_is_unsupported(torch, ctx):
    from paper_2210_12212_amd import IhsbinError
    M = W.csr_zipf(100, 400, 5, seed=4, dtype=np.float32)
    B = np.ones((100, 1), dtype=np.float32)
    with pytest.raises(IhsbinError) as e:
        ctx.solve_path(csr_dev(torch, M), dev(torch, B), [1.0], sketch="countsketch", m=50)
    assert e.value.status == -7


# ---------------------------------------------------------------- sketched Gram
@pytest.mark.parametrize("m,d", [(3000, 300), (700, 129), (5000, 64)])
def test_gram_precisions(torch, ctx, m, d):
    # FP64: the product itself; split BF16: within 1e-5 of sqrt(G_ii G_jj)
    r = np.random.default_rng(m + d)
    SA = r.standard_normal((m, d)) * np.exp(-np.arange(d) / 50.0)
    ref = SA.T @ SA
    low = np.tril_indices(d)
    G64 = ctx.gram(dev(torch, SA), "f64").cpu().numpy()
    np.testing.assert_allclose(G64[low], ref[low], rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    Gb = ctx.gram(dev(torch, SA), "bf16x3").cpu().numpy()
    scale = np.sqrt(np.outer(np.diag(ref), np.diag(ref)))
    assert (np.abs(Gb - ref)[low] <= 1e-5 * scale[low]).all()


@pytest.mark.parametrize("kind", ["srht", "countsketch"])
def test_path_with_bf16x3_gram(torch, ctx, kind):
    # the factor of a Gram accurate to ~1e-6 is a fixed SPD preconditioner:
    # the path converges to the same solution
    A = W.dense_decay(4000, 200, seed=91, dtype=np.float32)
    B, _ = W.rhs(A, 2, 0.1, seed=92)
    lams = W.lambda_grid(1e-3, 1e2, 13)
    X, rep = ctx.solve_path(dev(torch, A), dev(torch, B), lams, sketch=kind, m=100, seed=93,
                            gram_prec=1, tol=1e-9)
    assert rep["status"] == 0, rep
    err = direct.rel_err(X.cpu().numpy(), direct.ridge_path(A, B, lams))
    assert err.max() <= 1e-6, err


def test_path_refined_centres(torch, ctx):
    # the remark after Theorem 1: centres shifted by sigma_d^2; the same fixed
    # point, the oracle's centres, and no more steps than the plain centres
    r = np.random.default_rng(17)
    n, d = 4000, 120
    U, _ = np.linalg.qr(r.standard_normal((n, d)))
    A = (U * np.sqrt(np.geomspace(0.3, 300.0, d))).astype(np.float64)
    B = A @ r.standard_normal((d, 2)) + 0.1 * r.standard_normal((n, 2))
    s = float(np.linalg.eigvalsh(A.T @ A)[0])
    lams = W.lambda_grid(1e-2, 1e2, 25)
    out = {}
    for sd2 in (0.0, s):
        path, rep = ctx.path_build(dev(torch, A), dev(torch, B), lams[0], lams[-1], sketch="srht",
                                   m=1000, seed=5, sigma_d2=sd2)
        X = path.eval(lams).cpu().numpy()
        iv = path.intervals()
        path.free()
        _check_path(X, A, B, lams)
        grid, c = ihs_bin.plan(lams[0], lams[-1], len(iv["lam0"]), sigma_d2=sd2)
        np.testing.assert_allclose(iv["lam0"], c, rtol=1e-12)
        out[sd2] = rep["k_sum"]
    assert out[s] <= out[0.0], out


@pytest.mark.parametrize("prec,q,splits", [("f64", 1, 1), ("f64", 3, 4), ("f64", 7, 16),
                                           ("f64", 0, 0), ("f32", 2, 8), ("f32", 5, 1),
                                           ("f32", 0, 0)])
@pytest.mark.parametrize("w", [5, 40, 161])
def test_ata_forced_tilings(torch, ctx, prec, q, splits, w):
    # every tiling the tuner may pick computes the same product: FP64 to
    # rounding, FP32 (columns scaled by powers of two) to FP32 accuracy; the
    # columns differ in scale by 2^200 to exercise the scaling
    r = np.random.default_rng(w + q)
    A = r.standard_normal((5000, 120)).astype(np.float32)
    U = r.standard_normal((120, w)) * (2.0 ** (200 * (np.arange(w) % 3 - 1)))[None, :]
    Wg = ctx.ata_apply_tiled(dev(torch, A), dev(torch, U), prec, q, splits).cpu().numpy()
    A64 = A.astype(np.float64)
    ref = A64.T @ (A64 @ U)
    tol = 1e-12 if prec == "f64" else 2e-5
    colmax = np.abs(ref).max(axis=0)
    assert np.all(np.abs(Wg - ref) <= tol * colmax[None, :]), np.abs((Wg - ref) / colmax).max()
