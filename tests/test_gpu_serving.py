"""Serving: concurrent builds on one device give the results each build gives
alone, admission keeps the admitted memory estimates within the budget, and
the footprint estimate bounds what a build really allocates."""
import numpy as np
import pytest

import workloads as W
from oracle import direct

pytestmark = pytest.mark.gpu

TOL_PATH = 1e-6


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def csr_dev(torch, M):
    from paper_2210_12212_amd import CsrInput
    return CsrInput(dev(torch, M.row_ptr), dev(torch, M.col_idx), dev(torch, M.vals), M.n, M.d)


# (kind, n, d, K, sketch, dtype, lam range, extra options)
REQUESTS = [
    ("dense", 6000, 256, 2, "srht", np.float32, (1e-3, 1e1), {}),
    ("dense", 3000, 128, 1, "gaussian", np.float64, (1e-2, 1e2), {}),
    ("csr", 20000, 300, 3, "countsketch", np.float32, (1e-2, 1e2), {}),
    ("dense", 9000, 512, 1, "srht", np.float32, (1e-4, 1e1), dict(gram_prec=1)),
    ("dense", 4000, 200, 4, "sjlt", np.float64, (1e-3, 1e1), dict(sjlt_s=2)),
    ("dense", 5000, 96, 1, "countsketch", np.float32, (1e-3, 1e2), dict(adaptive_m=2, m=16)),
    ("dense", 300, 1200, 1, "srht", np.float32, (1e-2, 1e1), {}),   # n < d: dual
    ("dense", 7000, 160, 2, "gaussian", np.float32, (1e-3, 1e1), dict(adaptive_m=0, m=640)),
]


def _make(torch, i, req):
    kind, n, d, K, sketch, dt, (lo, hi), extra = req
    r = np.random.default_rng(100 + i)
    if kind == "csr":
        A = W.csr_zipf(n, d, 12, seed=100 + i, dtype=dt)
        Ad = csr_dev(torch, A)
        B = r.standard_normal((n, K)).astype(dt)
    else:
        A = (r.standard_normal((n, d)) * (np.arange(d) + 1.0) ** -0.6).astype(dt)
        Ad = dev(torch, A)
        B = (A.astype(np.float64) @ r.standard_normal((d, K)) +
             0.1 * r.standard_normal((n, K))).astype(dt)
    lams = W.lambda_grid(lo, hi, 20)
    opts = dict(sketch=sketch, seed=7 + i, **extra)
    return A, Ad, B, dev(torch, B), lams, opts


def test_footprint_bounds_the_measured_peak(torch):
    from paper_2210_12212_amd import Context, build_footprint
    for i, req in enumerate(REQUESTS):
        A, Ad, B, Bd, lams, opts = _make(torch, i, req)
        ctx = Context(0)  # fresh: holds nothing before the build
        path, rep = ctx.path_build(Ad, Bd, lams[0], lams[-1], **opts)
        path.free()
        ctx.close()
        shape = (A.n, A.d) if hasattr(A, "row_ptr") else A.shape
        est = build_footprint(shape, B.shape[1], lams[0], lams[-1], csr=hasattr(A, "row_ptr"),
                              dtype=str(np.dtype(req[5])), **opts)
        assert rep["peak_bytes"] > 0
        assert est >= rep["peak_bytes"], (i, est, rep["peak_bytes"])


def test_served_results_match_alone_and_oracle(torch):
    from paper_2210_12212_amd import Context, Server
    inputs = [_make(torch, i, req) for i, req in enumerate(REQUESTS)]
    # alone: one build at a time on a plain context
    ctx = Context(0)
    alone = []
    for A, Ad, B, Bd, lams, opts in inputs:
        path, _ = ctx.path_build(Ad, Bd, lams[0], lams[-1], **opts)
        alone.append(path.eval(lams).cpu().numpy())
        path.free()
    ctx.close()
    # in the mix: all submitted at once to four workers
    srv = Server(0, workers=4)
    ids = [srv.submit(Ad, Bd, lams[0], lams[-1], **opts) for A, Ad, B, Bd, lams, opts in inputs]
    got = []
    infos = []
    for rid, (A, Ad, B, Bd, lams, opts) in zip(ids, inputs):
        path, info = srv.wait(rid)
        got.append(path.eval(lams).cpu().numpy())
        infos.append(info)
        path.free()
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(REQUESTS) and st["max_concurrent"] >= 2
    assert st["max_inflight_bytes"] <= st["budget"]
    for i, (req, (A, Ad, B, Bd, lams, opts)) in enumerate(zip(REQUESTS, inputs)):
        # every kernel sums in a fixed order: the same bits alone and in the mix
        np.testing.assert_array_equal(got[i], alone[i])
        if req[1] < req[2]:
            ref = direct.ridge_path_dual(A, B, lams)
        else:
            ref = direct.ridge_path(A, B, lams)
        err = direct.rel_err(got[i], ref)
        assert err.max() <= TOL_PATH, (i, err.max())
        assert infos[i]["status"] == 0 and infos[i]["ms_build"] > 0
        assert infos[i]["ms_total"] >= infos[i]["ms_queue"]


def test_admission_respects_the_budget(torch):
    from paper_2210_12212_amd import Server, IhsbinError, build_footprint
    inputs = [_make(torch, i, req) for i, req in enumerate(REQUESTS[:4])]
    fps = []
    for (A, Ad, B, Bd, lams, opts), req in zip(inputs, REQUESTS):
        shape = (A.n, A.d) if hasattr(A, "row_ptr") else A.shape
        fps.append(build_footprint(shape, B.shape[1], lams[0], lams[-1],
                                   csr=hasattr(A, "row_ptr"), dtype=str(np.dtype(req[5])), **opts))
    budget = int(max(fps) * 1.2)
    srv = Server(0, workers=4, hbm_budget=budget)
    ids = [srv.submit(Ad, Bd, lams[0], lams[-1], **opts) for A, Ad, B, Bd, lams, opts in inputs]
    for rid in ids:
        path, info = srv.wait(rid)
        path.free()
    st = srv.stats()
    assert st["max_inflight_bytes"] <= budget and st["completed"] == 4
    # a request above the budget is refused at submission
    A, Ad, B, Bd, lams, opts = _make(torch, 0, REQUESTS[0])
    small = Server(0, workers=1, hbm_budget=1 << 20)
    with pytest.raises(IhsbinError):
        small.submit(Ad, Bd, lams[0], lams[-1], **opts)
    small.close()
    srv.close()


def test_path_outlives_the_server_and_unknown_ids(torch):
    from paper_2210_12212_amd import Server, IhsbinError
    A, Ad, B, Bd, lams, opts = _make(torch, 1, REQUESTS[1])
    srv = Server(0, workers=2)
    rid = srv.submit(Ad, Bd, lams[0], lams[-1], **opts)
    path, info = srv.wait(rid)
    with pytest.raises(IhsbinError):
        srv.wait(rid)  # collected already
    # an uncollected request is finished and freed by close()
    srv.submit(Ad, Bd, lams[0], lams[-1], **opts)
    srv.close()
    X = path.eval(lams).cpu().numpy()
    path.free()
    err = direct.rel_err(X, direct.ridge_path(A, B, lams))
    assert err.max() <= TOL_PATH
