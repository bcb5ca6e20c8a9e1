"""The allocation-free evaluation entry point against ihsbin_path_eval: the
same path, the same lambdas, bit-identical output, on consecutive calls that
share the device's one scratch array (the second with fewer lambdas), across
two paths, and with its size limit and range check."""
import numpy as np
import pytest

import workloads as W
from oracle import direct

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def test_noalloc_eval_matches_eval(torch):
    from paper_2210_12212_amd import Context, IhsbinError
    dev = torch.device("cuda", 0)
    ctx = Context(0)
    A = W.dense_decay(1500, 70, seed=101)
    B, _ = W.rhs(A, 3, 0.1, seed=102)
    path, rep = ctx.path_build(torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev),
                               1e-3, 1e2, sketch="srht", m=200, seed=7)
    A2 = W.dense_decay(900, 40, seed=103, dtype=np.float32)
    B2, _ = W.rhs(A2, 1, 0.1, seed=104)
    path2, _ = ctx.path_build(torch.from_numpy(A2).to(dev), torch.from_numpy(B2).to(dev),
                              1e-2, 1e1, sketch="countsketch", m=80, seed=8)
    rng = np.random.default_rng(5)
    # two calls in a row, the second smaller; lambdas in any order, the grid
    # ends, interval boundaries and repeats included
    lam1 = np.concatenate([np.exp(rng.uniform(np.log(1e-3), np.log(1e2), 997)),
                           [1e-3, 1e2], path.intervals()["lo"], [0.5, 0.5]])
    lam2 = np.exp(rng.uniform(np.log(1e-3), np.log(1e2), 37))
    for lam in (lam1, lam2):
        ref = path.eval(lam)
        out = torch.full_like(ref, float("nan"))
        path.eval_noalloc(lam, out)
        assert torch.equal(out, ref)
        err = direct.rel_err(out.cpu().numpy(), direct.ridge_path(A, B, lam))
        assert err.max() <= 1e-6
    # another path on the same device uses the same scratch array; FP32 output
    lam3 = np.exp(rng.uniform(np.log(1e-2), np.log(1e1), 500))
    ref3 = path2.eval(lam3, dtype=torch.float32)
    out3 = torch.empty_like(ref3)
    path2.eval_noalloc(lam3, out3)
    assert torch.equal(out3, ref3)
    # and the first path again, after the second one overwrote the scratch
    ref2 = path.eval(lam2)
    out2 = torch.empty_like(ref2)
    path.eval_noalloc(lam2, out2)
    assert torch.equal(out2, ref2)
    # limits: more lambdas than the scratch holds, a lambda out of range
    import ctypes as C
    from paper_2210_12212_amd import _lib
    big = np.full(262145, 1.0)
    small = torch.empty((1, path.d, path.K), dtype=torch.float64, device=dev)
    # rejected on its size before anything is written
    rc = _lib.lib().ihsbin_path_eval_noalloc(path._h, big.ctypes.data_as(C.POINTER(C.c_double)),
                                             len(big), C.c_void_p(small.data_ptr()), path.K,
                                             _lib.F64)
    assert rc == _lib.EINVAL
    with pytest.raises(IhsbinError) as e:
        path.eval_noalloc([1e3], torch.empty((1, path.d, path.K), dtype=torch.float64, device=dev))
    assert e.value.status == -6
    path.free()
    path2.free()
    ctx.close()
