"""Parity at the benchmarked sizes, in the launch configuration bench.py
times (the same tiles, columns, chunks and launches):

* one source iteration (sweep of every (cell, direction, band), plain
  scheme) of the 256 x 256 heat-source square, 128 directions, 20 bands,
  from a seeded anisotropic state, FP32 and FP64, element by element against
  the oracle's sweep of the same state;
* one explicit step of the 64^3 laser cube, 128 directions, 40 bands, MC
  limiter, FP32, element by element against the oracle's step;
* one source iteration of the 48^3 porous cube (40 bands, 96 directions,
  pores, per-cell scattering rates), FP32 and FP64, element by element
  against the oracle's sweep;
* one source iteration of the full batch of 64 porous films (sides 32 to
  256, 64 directions, 20 bands, minmod limiter, periodic with a drop along
  x, diffuse pores) swept in one problem, FP32 and FP64: the three smallest
  films and the largest element by element against the oracle's sweep of
  each film alone (the films are independent);
* one source iteration of the two-material interface workload (two
  128 x 256 halves of a 1 um square joined by the interfacial boundary
  condition, 128 directions, 20 bands per material), FP32 and FP64, element
  by element against the oracle's sweep of the same two-material geometry;
* the adjoint gradient d k_eff / d gamma of the 48^3 porous cube: FP64
  against central differences of the FP64 k_eff on 20 random cells, and
  the FP32 forward solve and adjoint behind autograd against FP64.

Bars as in the small-case parity tests: FP32 storage 1e-5, FP64 1e-11
(relative to the largest magnitude of the reference).
"""
import numpy as np
import pytest

import bte_inputs as I
import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_14181_amd import bte
    bte.load()
    return bte


def anisotropic_state(case, seed):
    """Equilibrium of a random temperature field plus 5 % anisotropic noise,
    rounded to FP32 (both sides start from exactly the same values)."""
    rng = np.random.default_rng(seed)
    T = rng.uniform(-1.0, 1.0, case.nc)
    base = case.C[None, :] / (4 * np.pi)
    e = np.empty((case.nc, case.na, case.nl), dtype=np.float32)
    scale = 0.05 * np.abs(base).max()
    step = 4096
    for c0 in range(0, case.nc, step):
        c1 = min(case.nc, c0 + step)
        blk = T[c0:c1, None, None] * base[None, :, :] + scale * rng.standard_normal((c1 - c0, case.na, case.nl))
        e[c0:c1] = blk.astype(np.float32)
    if case.solid is not None:
        e[case.solid == 0] = 0.0
    return e.reshape(-1)


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


_SWEEP = {}


def sweep_reference():
    if "ref" not in _SWEEP:
        cfg = I.square2d_source_case()
        case = O.Case(cfg["geometry"], cfg["material"], P=cfg["P"])
        e0 = anisotropic_state(case, 101)
        e1, st = O.steady(case, scheme=0, tol_T=0.0, tol_q=0.0, max_iter=1, e=e0.astype(np.float64))
        assert st["iters"] == 1
        _SWEEP["ref"] = (cfg, e0, e1)
    return _SWEEP["ref"]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_full_size_sweep_matches_oracle(B, prec):
    cfg, e0, e1 = sweep_reference()
    p = B.F32 if prec == "f32" else B.F64
    prob = B.Problem(cfg["geometry"], cfg["material"], dict(precision=p, scheme=B.SEQUENTIAL, limiter=B.LIM_NONE,
                                                            max_iter=1, residual_temp=0.0, residual_flux=0.0))
    prob.set_fields(torch.as_tensor(cfg["P"], device="cuda"), None)
    e = torch.as_tensor(e0, device="cuda").to(prob.dtype)
    st = prob.steady_solve(e, init=False, allow_not_converged=True)
    assert st["iters"] == 1 and st["updates"] == prob.n_unknowns
    g = e.double().cpu().numpy()
    del e, prob
    torch.cuda.empty_cache()
    err = rel(g, e1)
    print(prec, "full-size sweep rel err", err)
    assert err < (1e-5 if p == B.F32 else 1e-11), err


def test_full_size_transient_step_matches_oracle(B):
    cfg = I.cube3d_laser_case()
    case = O.Case(cfg["geometry"], cfg["material"], P=cfg["P"], limiter=O.LIM_MC)
    e0 = anisotropic_state(case, 202)
    prob = B.Problem(cfg["geometry"], cfg["material"], dict(precision=B.F32, limiter=B.LIM_MC, dt=cfg["dt"]))
    prob.set_fields(torch.as_tensor(cfg["P"], device="cuda"), None)
    e = torch.as_tensor(e0, device="cuda")
    t0 = 18e-12   # on the rising edge of the pulse
    prob.transient_step(e, 1, t0, cfg["pulse"])
    g = e.cpu().numpy()
    del e, prob
    torch.cuda.empty_cache()
    ref, _ = O.transient(case, e0.astype(np.float64), 1, cfg["dt"], t0, cfg["pulse"])
    # compare in slabs (the full state is 1.3e9 values)
    err = 0.0
    n = ref.size
    step = 1 << 26
    den = float(np.abs(ref).max())
    for i in range(0, n, step):
        err = max(err, float(np.abs(g[i:i + step].astype(np.float64) - ref[i:i + step]).max()) / den)
    print("full-size transient step rel err", err)
    assert err < 1e-5, err


_POROUS = {}


def porous_reference():
    """One plain source iteration of the 48^3 porous cube (gamma field, 40
    bands, 96 directions) from a seeded anisotropic state, by the oracle."""
    if "ref" not in _POROUS:
        cfg = I.porous3d_adjoint_case()
        case = O.Case(cfg["geometry"], cfg["material"], gamma=cfg["gamma"])
        e0 = anisotropic_state(case, 303)
        e1, st = O.steady(case, scheme=0, tol_T=0.0, tol_q=0.0, max_iter=1, e=e0.astype(np.float64))
        assert st["iters"] == 1
        _POROUS["ref"] = (cfg, e0, e1)
    return _POROUS["ref"]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_full_size_porous3d_sweep_matches_oracle(B, prec):
    """The 3D steady sweep at the porous-cube size, in the tile shape the
    library chooses for it (periodic x, y and z, spherical pores, per-cell
    scattering rates), element by element against the oracle's sweep."""
    cfg, e0, e1 = porous_reference()
    p = B.F32 if prec == "f32" else B.F64
    prob = B.Problem(cfg["geometry"], cfg["material"], dict(precision=p, scheme=B.SEQUENTIAL, limiter=B.LIM_NONE,
                                                            max_iter=1, residual_temp=0.0, residual_flux=0.0))
    prob.set_fields(None, torch.as_tensor(cfg["gamma"], device="cuda"))
    e = torch.as_tensor(e0, device="cuda").to(prob.dtype)
    st = prob.steady_solve(e, init=False, allow_not_converged=True)
    assert st["iters"] == 1
    g = e.double().cpu().numpy()
    del e, prob
    torch.cuda.empty_cache()
    err = rel(g, e1)
    print(prec, "porous 48^3 sweep rel err", err)
    assert err < (1e-5 if p == B.F32 else 1e-11), err


_BATCH = {}


def batch_reference():
    if "ref" not in _BATCH:
        cfg = I.porous2d_batch_case()
        films, mat = cfg["films"], cfg["material"]
        sizes = [int(np.prod(g["n"])) for g in films]
        order = np.argsort(sizes, kind="stable")
        pick = sorted(set(order[:3].tolist() + [int(order[-1])]))
        ref = {}
        for f in pick:
            case = O.Case(films[f], mat, limiter=O.LIM_MINMOD)
            e0 = anisotropic_state(case, 300 + f)
            e1, st = O.steady(case, scheme=0, tol_T=0.0, tol_q=0.0, max_iter=1, e=e0.astype(np.float64))
            assert st["iters"] == 1
            ref[f] = (e0, e1)
        _BATCH["ref"] = (cfg, sizes, ref)
    return _BATCH["ref"]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_full_size_batch_films_match_oracle(B, prec):
    """The batched-film sweep at its benchmarked size and launch shape."""
    cfg, sizes, ref = batch_reference()
    p = B.F32 if prec == "f32" else B.F64
    prob = B.Problem(cfg["films"], cfg["material"], dict(precision=p, scheme=B.SEQUENTIAL, limiter=B.LIM_MINMOD,
                                                         max_iter=1, residual_temp=0.0, residual_flux=0.0))
    nk = prob.n_dirs * prob.n_bands
    start = np.concatenate([[0], np.cumsum(sizes)]) * nk
    e = prob.zeros()
    for f, (e0, _) in ref.items():
        e[start[f]:start[f + 1]] = torch.as_tensor(e0, device="cuda").to(prob.dtype)
    st = prob.steady_solve(e, init=False, allow_not_converged=True)
    assert st["iters"] == 1
    for f, (_, e1) in ref.items():
        g = e[start[f]:start[f + 1]].double().cpu().numpy()
        err = rel(g, e1)
        print(prec, "film", f, "cells", sizes[f], "rel err", err)
        assert err < (1e-5 if p == B.F32 else 1e-11), (f, err)
    del e, prob
    torch.cuda.empty_cache()


def _keff_solve(B, prob, gamma, e_start=None):
    prob.set_fields(None, torch.as_tensor(gamma, device="cuda"))
    e = prob.zeros() if e_start is None else e_start.clone()
    st = prob.steady_solve(e, init=e_start is None)
    assert st["converged"], st
    return prob.keff(e).item(), e


def test_full_size_adjoint_against_central_differences(B):
    """d k_eff / d gamma of the 48^3 porous cube.

    * FP64 adjoint against central differences of the FP64 k_eff on 20
      random solid cells (h = 1e-4 gamma_c, at least 1e6 1/s).  One cell
      moves k_eff by ~1e-9 of itself, so the difference quotient of two
      solves converged to eps_T 1e-13 resolves the derivative only to
      ~1e-13 k / h, about 5e-5 of max |grad| here; the FD bar is 1e-4 of
      max |grad| (measured worst 9.6e-5).
    * FP32 forward solve and FP32 adjoint behind KeffSteady against the
      FP64 adjoint, every cell: 5e-5 of max |grad| (measured 3.3e-5).  The
      gradient weighs e - e0 (the non-equilibrium part of the forward
      state), a small difference of FP32-stored values, and its error does
      not move with the adjoint tolerance (3.0e-5 at residual 2e-7, 3.3e-5
      at 1e-6, 3.9e-5 at 3e-6): it is the FP32 forward state's, not the
      adjoint iteration's.  k_eff itself agrees to 1e-5 (measured 5e-7)."""
    cfg = I.porous3d_adjoint_case()
    g, m, gam0 = cfg["geometry"], cfg["material"], cfg["gamma"]
    ctl = dict(scheme=B.SYNTHETIC, limiter=B.LIM_NONE, adjoint=True, max_iter=5000, cg_rtol=1e-12,
               cg_max_iter=2000)
    solid = np.asarray(g["solid"]).astype(bool)
    p64 = B.Problem(g, m, dict(ctl, precision=B.F64, residual_temp=1e-13, residual_flux=1e-12))
    k64, e64 = _keff_solve(B, p64, gam0)
    grad64, st = p64.adjoint(e64)
    assert st["converged"], st
    grad64 = grad64.cpu().numpy()
    gmax = np.abs(grad64).max()
    assert np.all(grad64[~solid] == 0.0)
    rng = np.random.default_rng(44)
    worst = 0.0
    for c in rng.choice(np.flatnonzero(solid), 20, replace=False):
        h = 1e-4 * max(gam0[c], 1e10)
        ks = []
        for sg in (1, -1):
            g2 = gam0.copy()
            g2[c] += sg * h
            ks.append(_keff_solve(B, p64, g2, e64)[0])
        fd = (ks[0] - ks[1]) / (2 * h)
        worst = max(worst, abs(fd - grad64[c]) / gmax)
        print("cell", c, "fd", fd, "adjoint FP64", grad64[c])
    print("worst FD deviation / max |grad|", worst)
    assert worst <= 1e-4, worst
    del p64, e64
    torch.cuda.empty_cache()
    # FP32 forward (to eps_T 1e-7) and FP32 adjoint (to a relative residual
    # of 1e-6, reached in ~50 sweeps; its FP32 floor is ~2e-7) behind autograd
    p32 = B.Problem(g, m, dict(ctl, precision=B.F32, residual_temp=1e-7, residual_flux=1e-6))
    gamma = torch.as_tensor(gam0, device="cuda").requires_grad_(True)
    k32 = B.KeffSteady.apply(gamma, p32, None)
    p32.set_control(residual_temp=1e-6)
    k32.sum().backward()
    grad32 = gamma.grad.cpu().numpy()
    assert np.all(grad32[~solid] == 0.0)
    err = float(np.abs(grad32 - grad64).max() / gmax)
    print("k_eff FP32", k32.item(), "FP64", k64, "grad FP32 vs FP64", err)
    assert abs(k32.item() / k64 - 1) < 1e-5 and err < 5e-5, (k32.item(), k64, err)


_IFACE = {}


def interface_reference():
    """The interface workload as the oracle's one two-material geometry, a
    seeded anisotropic FP32 state and the oracle's sweep of it; cmap[i] is
    the device cell of oracle cell i."""
    if "ref" not in _IFACE:
        cfg = I.interface2d_case()
        gA, gB = cfg["geometries"]
        nA, nB, ny = gA["n"][0], gB["n"][0], gA["n"][1]
        n = nA + nB
        mat = np.zeros((ny, n), dtype=np.int32)
        mat[:, nA:] = 1
        gu = dict(dim=2, n=[n, ny, 1], len=[gA["len"][0] + gB["len"][0], gA["len"][1], 1.0],
                  bc=[gA["bc"][0], gB["bc"][1]] + gA["bc"][2:], bcT=[gA["bcT"][0], gB["bcT"][1]] + gA["bcT"][2:],
                  pdT=[0.0, 0.0, 0.0], solid=None, pore_bc=gA["pore_bc"], mat=mat.reshape(-1))
        q = cfg["interfaces"][0]
        beta = np.zeros((2, 2, len(q["beta_ab"])))
        beta[0, 1], beta[1, 0] = q["beta_ab"], q["beta_ba"]
        case = O.Case(gu, cfg["materials"], beta=beta)
        rng = np.random.default_rng(102)
        T = rng.uniform(-1.0, 1.0, case.nc)
        C4 = case.C.reshape(case.nmat, case.nl)[case.mat] / (4 * np.pi)          # [nc, nl]
        scale = 0.05 * np.abs(C4).max()
        e0 = np.empty((case.nc, case.na, case.nl), dtype=np.float32)
        for c0 in range(0, case.nc, 4096):
            c1 = min(case.nc, c0 + 4096)
            blk = T[c0:c1, None, None] * C4[c0:c1, None, :] + scale * rng.standard_normal((c1 - c0, case.na, case.nl))
            e0[c0:c1] = blk.astype(np.float32)
        e0 = e0.reshape(-1)
        e1, st = O.steady(case, scheme=0, tol_T=0.0, tol_q=0.0, max_iter=1, e=e0.astype(np.float64))
        assert st["iters"] == 1
        cmap = np.empty(n * ny, dtype=np.int64)
        iy, ix = np.divmod(np.arange(n * ny), n)
        cmap[:] = np.where(ix < nA, ix + nA * iy, nA * ny + (ix - nA) + nB * iy)
        _IFACE["ref"] = (cfg, case, cmap, e0, e1)
    return _IFACE["ref"]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_full_size_interface_sweep_matches_oracle(B, prec):
    cfg, case, cmap, e0, e1 = interface_reference()
    p = B.F32 if prec == "f32" else B.F64
    prob = B.Problem(cfg["geometries"], cfg["materials"],
                     dict(precision=p, scheme=B.SEQUENTIAL, limiter=B.LIM_NONE, max_iter=1, residual_temp=0.0,
                          residual_flux=0.0),
                     geo_mat=cfg["geo_mat"], interfaces=cfg["interfaces"])
    prob.set_persistent(True)   # the form the bench keeps
    ed = np.empty_like(e0.reshape(case.nc, -1))
    ed[cmap] = e0.reshape(case.nc, -1)
    e = torch.as_tensor(ed.reshape(-1), device="cuda").to(prob.dtype)
    del ed
    st = prob.steady_solve(e, init=False, allow_not_converged=True)
    assert st["iters"] == 1 and st["updates"] == prob.n_unknowns
    g = e.double().cpu().numpy().reshape(case.nc, -1)[cmap].reshape(-1)
    del e, prob
    torch.cuda.empty_cache()
    err = rel(g, e1)
    print(prec, "full-size interface sweep rel err", err)
    assert err < (1e-5 if p == B.F32 else 1e-11), err

