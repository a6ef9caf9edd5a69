"""bte_moments_static, the entry point that allocates nothing (its FP64
moment partials live in the library's static device scratch), called
through the C ABI against bte_moments on the same state: bit-identical T,
T_L and q on two calls in a row, the second on a smaller problem (the
scratch keeps the first call's contents), and the size limit."""
import ctypes as C

import numpy as np
import pytest

import bte_inputs as I
from tests.helpers import small_cases

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_14181_amd import bte
    bte.load()
    return bte


def _call(B, fn, prob, e, fill=None):
    n = prob.n_cells
    outs = [torch.full((n,), fill if fill is not None else 0.0, dtype=torch.float64, device="cuda"),
            torch.full((n,), fill if fill is not None else 0.0, dtype=torch.float64, device="cuda"),
            torch.full((3 * n,), fill if fill is not None else 0.0, dtype=torch.float64, device="cuda")]
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = fn(prob._h, C.c_void_p(e.data_ptr()), *[C.c_void_p(t.data_ptr()) for t in outs], stream)
    torch.cuda.synchronize()
    return st, outs


def _state(prob, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    return (torch.randn(prob.n_unknowns, generator=g, dtype=torch.float64) * 10.0).to("cuda", prob.dtype)


def test_static_moments_match_workspace_moments_twice(B):
    lib = B.load()
    big = I.square2d_source_case(n=96, n_bands=6, n_theta=2, n_phi=2)
    p1 = B.Problem(big["geometry"], big["material"], dict(precision=B.F32))
    g, m, P, gam = small_cases()["box3d"]
    p2 = B.Problem(g, m, dict(precision=B.F64))
    p2.set_fields(None, torch.as_tensor(gam, device="cuda"))
    assert p2.n_cells < p1.n_cells
    for prob, seed in ((p1, 1), (p2, 2)):
        e = _state(prob, seed)
        st_ws, ref = _call(B, lib.bte_moments, prob, e)
        st_st, got = _call(B, lib.bte_moments_static, prob, e, fill=float("nan"))
        assert st_ws == 0 and st_st == 0, (st_ws, st_st, lib.bte_last_error(prob._h))
        for r, x in zip(ref, got):
            assert torch.equal(r, x), float((r - x).abs().max())


def test_static_moments_reject_too_many_cells(B):
    lib = B.load()
    limit = 838860
    n = limit + 1
    geo = dict(dim=1, n=[n, 1, 1], len=[n * 1e-9, 1.0, 1.0], bc=[I.BC_PERIODIC] * 2 + [I.BC_SPECULAR] * 4,
               bcT=[300.0] * 6, pdT=[0.0] * 3, solid=None, pore_bc=I.BC_DIFFUSE)
    mat = dict(C=np.array([1.66e6]), v=np.array([3000.0]), tau=np.array([1e-11]), n_theta=1, n_phi=1, Tref=300.0)
    prob = B.Problem(geo, mat, dict(precision=B.F32))
    e = prob.zeros()
    st, outs = _call(B, lib.bte_moments_static, prob, e, fill=-1.0)
    assert st == B.BTE_ERR_ARG
    assert all(bool((t == -1.0).all()) for t in outs)
    # the workspace form has no such limit
    st, _ = _call(B, lib.bte_moments, prob, e)
    assert st == 0
