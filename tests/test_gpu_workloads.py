"""GPU parity on the configured workloads at their full sizes.

The path is built in the configuration bench.py times and every lambda is
compared with the oracle at 1e-6 relative error, through the
eigendecomposition of G = A^T A (the closed form of Section 2.1; pinned
against the per-lambda Cholesky solve in the CPU tests).
"""
import time

import numpy as np
import pytest

import workloads as W
from oracle import direct

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


def _to_dev(torch, p):
    from paper_2210_12212_amd import CsrInput
    dev = torch.device("cuda", 0)
    if isinstance(p.A, W.CsrMatrix):
        A = CsrInput(torch.from_numpy(p.A.row_ptr).to(dev), torch.from_numpy(p.A.col_idx).to(dev),
                     torch.from_numpy(p.A.vals).to(dev), p.A.n, p.A.d)
    else:
        A = torch.from_numpy(p.A).to(dev)
    return A, torch.from_numpy(p.B).to(dev)


def _reference(p):
    # one eigendecomposition of G serves every lambda (O(d^3) once, O(d^2 K)
    # per lambda); progress is printed so a long oracle step is visibly alive
    t0 = time.time()
    G = direct.gram(p.A)
    C = direct.atb(p.A, p.B)
    print(f"  oracle: G and A^T B in {time.time() - t0:.1f}s", flush=True)
    ev, V = direct.eig_of_gram(G)
    print(f"  oracle: eigendecomposition in {time.time() - t0:.1f}s", flush=True)
    return direct.solve_from_eig(ev, V, C, p.lambdas)


def _check_every_lambda(p, X, tol=1e-6, ref=None):
    ref = _reference(p) if ref is None else ref
    err = direct.rel_err(X, ref)
    print(f"{p.name}: every lambda, max rel err {err.max():.3e}", flush=True)
    assert err.max() <= tol, err
    return err


def test_dense_exp300_131072x2048_srht_as_benched(torch, ctx):
    p = W.make("dense_exp300_131072x2048")
    A, B = _to_dev(torch, p)
    X, rep = ctx.solve_path(A, B, p.lambdas, sketch=p.sketch, m=p.m, seed=p.sketch_seed, tol=1e-7,
                            rate_target=0.5, lanczos_steps=4)
    assert rep["status"] == 0 and rep["n_unconverged"] == 0, rep
    _check_every_lambda(p, X.cpu().numpy())


@pytest.mark.timeout(600)
def test_csr_zipf_1048576x8192_countsketch(torch, ctx):
    p = W.make("csr_zipf_1048576x8192")
    A, B = _to_dev(torch, p)
    X, rep = ctx.solve_path(A, B, p.lambdas, sketch=p.sketch, m=p.m, seed=p.sketch_seed, tol=1e-7)
    assert rep["status"] == 0, rep
    _check_every_lambda(p, X.cpu().numpy())


@pytest.fixture(scope="module")
def invsqrt_full():
    p = W.make("dense_invsqrt_262144x4096_k64")
    cache = {}

    def ref():
        if "X" not in cache:
            cache["X"] = _reference(p)
        return cache["X"]
    return p, ref


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["bf16", "f64"])
def test_dense_invsqrt_262144x4096_k64_full_size(torch, ctx, invsqrt_full, prec):
    # the matrix-valued workload at its full size (Section 5.3, 64 right-hand
    # sides), Gaussian sketch from m0 = 2048, with the sketch product on the
    # BF16 matrix cores (as bench.py times it) and in FP64
    p, ref = invsqrt_full
    A, B = _to_dev(torch, p)
    X, rep = ctx.solve_path(A, B, p.lambdas, sketch=p.sketch, m=p.m, seed=p.sketch_seed, tol=1e-7,
                            rate_target=0.5, lanczos_steps=4,
                            sketch_prec={"f64": 0, "bf16": 1}[prec])
    assert rep["status"] == 0, rep
    del A, B
    print(f"invsqrt {prec}: m_used={rep['m_used']} k_max={rep['k_max_used']} "
          f"ms={rep['ms_total']:.0f}", flush=True)
    _check_every_lambda(p, X.cpu().numpy(), ref=ref())


def test_dense_invsqrt_k64_reduced_n(torch, ctx):
    # 64 right-hand sides (matrix-valued problem, Section 5.3) on n = 16384 rows
    p = W.make("dense_invsqrt_262144x4096_k64", n=16384, d=1024)
    A, B = _to_dev(torch, p)
    X, rep = ctx.solve_path(A, B, p.lambdas, sketch=p.sketch, m=p.m // 4, seed=p.sketch_seed, tol=1e-7)
    assert rep["status"] == 0, rep
    _check_every_lambda(p, X.cpu().numpy())


def test_strided_rows_and_rhs(torch, ctx):
    # A given as a column slice of a wider matrix (row stride > d), B likewise
    wide = W.dense_decay(3000, 80, seed=3)
    Bw, _ = W.rhs(wide, 5, 0.1, seed=4)
    dev = torch.device("cuda", 0)
    At = torch.from_numpy(wide).to(dev)[:, :64]
    Bt = torch.from_numpy(Bw).to(dev)[:, :2]
    lams = W.lambda_grid(1e-2, 1e2, 13)
    X, rep = ctx.solve_path(At, Bt, lams, sketch="srht", m=256, seed=1)
    A = np.ascontiguousarray(wide[:, :64])
    B = np.ascontiguousarray(Bw[:, :2])
    err = direct.rel_err(X.cpu().numpy(), direct.ridge_path(A, B, lams))
    assert err.max() <= 1e-6
