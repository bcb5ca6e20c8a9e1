"""GPU checks of the boundary calls added around the path: the integer draws
(device against the library's host computation and the oracle), the
column-major copy of a CSR matrix against SciPy's stable transpose, CSR
inputs with duplicate entries and empty rows, the Gaussian sketch of a CSR
matrix, the report's error estimate and byte count, and the random
over-determined experiment of Section 6.1 at its printed size."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import direct, ihs_bin, rng, sketch

pytestmark = pytest.mark.gpu


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


def messy_csr(n, d, per, seed, dtype=np.float32):
    """A Zipf CSR matrix with every 7th row emptied and, in every 5th
    non-empty row, its first column repeated once (a duplicate entry that the
    products must sum)."""
    M = W.csr_zipf(n, d, per, seed=seed, dtype=dtype)
    rp = M.row_ptr.astype(np.int64)
    cols, vals, ptr = [], [], [0]
    r = np.random.default_rng(seed + 1)
    for i in range(n):
        c = list(M.col_idx[rp[i]:rp[i + 1]])
        v = list(M.vals[rp[i]:rp[i + 1]])
        if i % 7 == 3:
            c, v = [], []
        elif i % 5 == 0 and c:
            c.append(c[0])
            v.append(dtype(r.standard_normal()))
        cols += c
        vals += v
        ptr.append(len(cols))
    return W.CsrMatrix(n, d, np.asarray(ptr, dtype=np.int32), np.asarray(cols, dtype=np.int32),
                       np.asarray(vals, dtype=dtype))


# ---------------------------------------------------------------- draws
@pytest.mark.parametrize("kind,n,m,s", [("countsketch", 5000, 333, 1), ("sjlt", 4099, 64, 4),
                                        ("srht", 3000, 700, 1), ("countsketch", 1, 3, 1)])
def test_device_host_oracle_draws_agree_bitwise(torch, ctx, kind, n, m, s):
    from paper_2210_12212_amd import sketch_indices_host
    idx_d, sg_d = ctx.sketch_indices_device(4242, kind, n, m, s)
    idx_h, sg_h = sketch_indices_host(4242, kind, n, m, s)
    assert np.array_equal(idx_d.cpu().numpy(), idx_h)
    assert np.array_equal(sg_d.cpu().numpy(), sg_h)
    if kind == "srht":
        sg_o, rr_o, _ = rng.srht_draws(4242, n, m)
        assert np.array_equal(idx_h, rr_o) and np.array_equal(sg_h, sg_o)
    else:
        h, sg = rng.countsketch_draws(4242, n, m, s)
        assert np.array_equal(idx_h, h.reshape(-1)) and np.array_equal(sg_h, sg.reshape(-1))


# ------------------------------------------------------- column-major copy
@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("n,d,per", [(5000, 300, 9), (20000, 64, 20), (50, 1000, 3)])
def test_csc_copy_is_the_stable_transpose(torch, ctx, dt, n, d, per):
    M = messy_csr(n, d, per, seed=n + d, dtype=dt)
    cp, row, val = ctx.csr_transpose(csr_dev(torch, M))
    # SciPy's CSR -> CSC conversion walks the rows in order and appends each
    # entry to its column: the stable transpose, duplicates kept apart
    T = sp.csr_matrix((M.vals, M.col_idx, M.row_ptr), shape=(n, d)).tocsc()
    assert np.array_equal(cp.cpu().numpy(), T.indptr.astype(np.int32))
    assert np.array_equal(row.cpu().numpy(), T.indices.astype(np.int32))
    assert np.array_equal(val.cpu().numpy().view(np.uint8), T.data.astype(dt).view(np.uint8))


def test_csc_copy_of_full_size_zipf(torch, ctx):
    M = W.csr_zipf(1 << 20, 8192, 24, seed=1000, dtype=np.float32)
    cp, row, val = ctx.csr_transpose(csr_dev(torch, M))
    T = sp.csr_matrix((M.vals, M.col_idx, M.row_ptr), shape=(M.n, M.d)).tocsc()
    assert np.array_equal(cp.cpu().numpy(), T.indptr.astype(np.int32))
    assert np.array_equal(row.cpu().numpy(), T.indices.astype(np.int32))
    assert np.array_equal(val.cpu().numpy(), T.data)


# ------------------------------------------- duplicates and empty rows
@pytest.mark.parametrize("w", [1, 7, 70])
def test_ata_csr_duplicates_and_empty_rows(torch, ctx, w):
    M = messy_csr(6000, 250, 8, seed=w, dtype=np.float64)
    U = np.random.default_rng(w).standard_normal((250, w))
    Wg = ctx.ata_apply(csr_dev(torch, M), dev(torch, U)).cpu().numpy()
    ref = ihs_bin.Operator(M).AtA(U)
    np.testing.assert_allclose(Wg, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("kind", ["countsketch", "sjlt", "gaussian"])
def test_path_csr_duplicates_and_empty_rows(torch, ctx, kind):
    M = messy_csr(8000, 180, 7, seed=77)
    B, _ = W.rhs(M, 2, 0.1, seed=78)
    lams = W.lambda_grid(1e-2, 1e2, 19)
    X, rep = ctx.solve_path(csr_dev(torch, M), dev(torch, B), lams, sketch=kind, m=360, seed=3,
                            sjlt_s=2)
    assert rep["status"] == 0, rep
    err = direct.rel_err(X.cpu().numpy(), direct.ridge_path(M, B, lams))
    assert err.max() <= 1e-6, err


# ------------------------------------------------ Gaussian sketch of CSR
@pytest.mark.parametrize("m", [64, 300, 1000])
def test_gaussian_sketch_of_csr(torch, ctx, m):
    M = messy_csr(3000, 120, 5, seed=m)
    SA = ctx.sketch_apply(csr_dev(torch, M), "gaussian", m, 77).cpu().numpy()
    ref = sketch.apply("gaussian", M, 77, m)
    # the Gaussian entries go through device log/cos/sqrt: allow a few ulp
    np.testing.assert_allclose(SA, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


# ------------------------------------- Gram of a sparse (CSR) sketch
def _gram_parts_close(G, ref, d, tol=1e-12):
    """The lower triangle and the diagonal 64 x 64 tiles of G against ref."""
    scale = np.abs(ref).max()
    low = np.tril_indices(d)
    np.testing.assert_allclose(G[low], ref[low], rtol=tol, atol=tol * scale)
    for t0 in range(0, d, 64):
        t1 = min(d, t0 + 64)
        np.testing.assert_allclose(G[t0:t1, t0:t1], ref[t0:t1, t0:t1], rtol=tol, atol=tol * scale)


@pytest.mark.parametrize("kind,n,d,per,m,s", [
    ("countsketch", 20000, 3000, 9, 4000, 1),   # heavy columns (several chunks), three LDS ranges
    ("sjlt", 12000, 700, 6, 1200, 3),
    ("countsketch", 3000, 150, 5, 64, 1),       # m < d: every bucket holds many rows
])
def test_sketch_gram_of_csr_is_sparse_and_exact(torch, ctx, kind, n, d, per, m, s):
    # CountSketch / SJLT of a CSR matrix: the build keeps SA sparse and forms
    # (SA)^T SA from its entries; it must equal the Gram of the oracle's sketch
    M = messy_csr(n, d, per, seed=n % 97)
    G = ctx.sketch_gram(csr_dev(torch, M), kind, m, 123, sjlt_s=s).cpu().numpy()
    SA = sketch.apply(kind, M, 123, m, s=s)
    _gram_parts_close(G, SA.T @ SA, d)


def test_sketch_gram_dense_matches_gram_of_sketch(torch, ctx):
    # the dense path of the same call: the Gram of the library's own SA
    A = W.dense_decay(3000, 200, seed=8, dtype=np.float32)
    G = ctx.sketch_gram(dev(torch, A), "countsketch", 400, 5).cpu().numpy()
    SA = sketch.apply("countsketch", A, 5, 400)
    _gram_parts_close(G, SA.T @ SA, 200)


def test_sketch_gram_empty_columns(torch, ctx):
    # columns of A without entries give zero rows and columns of G
    M = W.csr_zipf(4000, 300, 4, seed=12, dtype=np.float32)
    keep = M.col_idx < 250           # columns 250.. have no entries
    rp = np.concatenate([[0], np.cumsum([keep[M.row_ptr[i]:M.row_ptr[i + 1]].sum()
                                         for i in range(M.n)])]).astype(np.int32)
    M2 = W.CsrMatrix(M.n, M.d, rp, M.col_idx[keep].copy(), M.vals[keep].copy())
    G = ctx.sketch_gram(csr_dev(torch, M2), "countsketch", 500, 9).cpu().numpy()
    SA = sketch.apply("countsketch", M2, 9, 500)
    ref = SA.T @ SA
    _gram_parts_close(G, ref, 300)
    for c in range(250, 300):        # their rows of the lower triangle are exactly zero
        assert not G[c, :c + 1].any()


# --------------------------------------------------------------- report
def test_report_estimate_and_bytes(torch, ctx):
    A = W.dense_decay(3000, 100, seed=5, dtype=np.float32)
    B, _ = W.rhs(A, 1, 0.1, seed=6)
    lams = W.lambda_grid(1e-3, 1e2, 31)
    X, rep = ctx.solve_path(dev(torch, A), dev(torch, B), lams, sketch="srht", m=200, seed=1,
                            tol=1e-8)
    assert rep["status"] == 0
    assert 0.0 < rep["est_rel_err"] <= 1e-8
    err = direct.rel_err(X.cpu().numpy(), direct.ridge_path(A, B, lams))
    assert err.max() <= 1e-6
    # every basis step reads A twice; the sketch and A^T B once more each
    abytes = 3000 * 100 * 4
    assert rep["bytes_moved"] >= abytes * (2 * rep["steps"] + 2)
    # k_max too small: the estimate says the tolerance was not met
    _, rep2 = ctx.solve_path(dev(torch, A), dev(torch, B), lams, sketch="srht", m=200, seed=1,
                             tol=1e-8, k_max=3)
    assert rep2["status"] == -5 and rep2["est_rel_err"] > 1e-8


def test_eval_rejects_bad_out(torch, ctx):
    A = W.dense_decay(500, 20, seed=8)
    B, _ = W.rhs(A, 2, 0.1, seed=9)
    path, _ = ctx.path_build(dev(torch, A), dev(torch, B), 0.1, 10.0, sketch="srht", m=64)
    with pytest.raises(ValueError):
        path.eval([1.0, 2.0], out=torch.empty((1, 20, 2), dtype=torch.float64, device="cuda:0"))
    with pytest.raises(ValueError):
        # every other block of a wider allocation: block stride 2 d K
        spaced = torch.empty((3, 20, 2), dtype=torch.float64, device="cuda:0")[::2]
        path.eval([1.0, 2.0], out=spaced)
    with pytest.raises(ValueError):
        path.eval([1.0, 2.0], out=torch.empty((2, 20, 2), dtype=torch.float64))
    # a row stride wider than K is allowed (ldx >= K)
    wide = torch.empty((2, 20, 5), dtype=torch.float64, device="cuda:0")[:, :, :2]
    ref = path.eval([1.0, 2.0])
    path.eval([1.0, 2.0], out=wide)
    assert torch.equal(wide, ref)
    path.free()


# --------------------------------------------- Section 6.1 random data
def test_ar1_random_experiment_every_lambda(torch, ctx):
    # n = 20000, d = 4000, m = 1600, lambda in [1, 100], SJLT of sparsity 1
    p = W.make("dense_ar1_20000x4000")
    X, rep = ctx.solve_path(dev(torch, p.A), dev(torch, p.B), p.lambdas, sketch=p.sketch, m=p.m,
                            seed=p.sketch_seed, tol=1e-8)
    assert rep["status"] == 0, rep
    err = direct.rel_err(X.cpu().numpy(), direct.ridge_path(p.A, p.B, p.lambdas))
    print(f"ar1: m_used={rep['m_used']} k_max={rep['k_max_used']} max_err={err.max():.2e}")
    assert err.max() <= 1e-6, err
