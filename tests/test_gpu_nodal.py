"""GPU nodal solver (trilinear finite elements, Galerkin coarsening, Jacobi,
CG bottom) against the oracle (oracle/nodal.py), through the C ABI."""

import numpy as np
import pytest
import torch

import oracle.nodal as ON
import workloads as W
from gpu_util import lib, rel_l2

TIGHT = 1e-12

UNEVEN32 = [((0, 0, 0), (15, 31, 31)), ((16, 0, 0), (31, 15, 31)), ((16, 16, 0), (31, 31, 15)),
            ((16, 16, 16), (31, 31, 31))]

CASES = [
    # name, n, boxes, periodic, min_bottom_edge
    ("dirichlet32_8boxes", 32, W.uniform_boxes(32, 16), (False, False, False), 4),
    ("dirichlet64_8boxes", 64, W.uniform_boxes(64, 32), (False, False, False), 4),
    ("periodic_xz32_uneven", 32, UNEVEN32, (True, False, True), 4),
    ("periodic_y32_one_box", 32, [W.domain_box(32)], (False, True, False), 2),
    ("all_periodic16_singular", 16, W.uniform_boxes(16, 8), (True, True, True), 4),
    ("dirichlet48_27boxes_bottom6", 48, W.uniform_boxes(48, 16), (False, False, False), 4),
]


def _inputs(n, boxes, per, seed=0):
    cfg = W.config_nodal(n, n, 1.0, per)
    f = cfg["rhs_unknowns"]
    if all(per):
        f = f - f.mean()
    return cfg["sigma_cells"], f


def _gpu(n, boxes, per, sigma, opts):
    P = lib()
    sm = P.MultiFab.from_numpy(boxes, W.scatter_cells(sigma, boxes), 0)
    return P.NodalMLMG(boxes, W.domain_box(n), per, sigma=sm, opts=opts)


def _nodal_mf(P, boxes, U, n, per, ng, fill=np.nan):
    G = W.nodes_from_unknowns(U, n, per)
    return P.MultiFab.from_numpy(boxes, W.scatter_nodes(G, boxes, ng, fill=fill), ng,
                                 ixtype=(1, 1, 1))


def _unknowns(mf, boxes, n, per):
    """Unknowns from a nodal MultiFab, checking that every copy of a node in
    every box array (ghosts included) holds the same value."""
    G = np.full(tuple([n + 1] * 3), np.nan)
    ng = mf.ngrow
    for (lo, hi), a in zip(boxes, mf.to_numpy()):
        sl = tuple(slice(lo[d], hi[d] + 2) for d in range(3))
        v = a[ng:a.shape[0] - ng, ng:a.shape[1] - ng, ng:a.shape[2] - ng] if ng else a
        seen = G[sl]
        m = ~np.isnan(seen)
        assert np.array_equal(seen[m], v[m]), "a node's copies differ between boxes"
        G[sl] = v
    return W.unknowns_from_nodes(G, per), G


@pytest.mark.gpu
@pytest.mark.parametrize("name,n,boxes,per,mbe", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("ng", [0, 1])
def test_nodal_apply_vs_oracle(name, n, boxes, per, mbe, ng):
    print(f"[nodal] apply {name} ng={ng}", flush=True)
    P = lib()
    sigma, _ = _inputs(n, boxes, per)
    s = _gpu(n, boxes, per, sigma, dict(min_bottom_edge=mbe))
    x = np.random.default_rng(3).standard_normal(W.nodal_unknown_shape(n, per))
    phi = _nodal_mf(P, boxes, x, n, per, ng)
    out = s.node_mf(ng, fill=np.nan)
    s.apply(phi, out)
    torch.cuda.synchronize()
    got, G = _unknowns(out, boxes, n, per)
    ref = ON.apply_nodal(ON.make_nodal_level(sigma, per), x)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    # wall nodes hold 0
    for d in range(3):
        if not per[d]:
            sl = [slice(None)] * 3
            sl[d] = 0
            assert np.all(G[tuple(sl)] == 0.0)
    s.close()


def _solve_pair(n, boxes, per, mbe, max_iter=100, tol=1e-10, opts=None):
    P = lib()
    sigma, f = _inputs(n, boxes, per)
    gopts = dict(bottom_rel_tol=TIGHT, min_bottom_edge=mbe, max_iter=max_iter)
    gopts.update(opts or {})
    s = _gpu(n, boxes, per, sigma, gopts)
    rhs = _nodal_mf(P, boxes, f, n, per, 0)
    phi = s.node_mf(1, fill=0.0)
    info = s.solve(phi, rhs, tol, history=True, raise_on_fail=False)
    torch.cuda.synchronize()
    got, _ = _unknowns(phi, boxes, n, per)
    ophi, oinfo = ON.nodal_solve(sigma, per, f, tol, opts=ON.NodalOpts(
        bottom_tol=TIGHT, min_bottom_cells=mbe, max_iter=max_iter))
    nl = s.num_levels()
    s.close()
    return info, got, oinfo, ophi, nl


@pytest.mark.gpu
@pytest.mark.parametrize("name,n,boxes,per,mbe", CASES, ids=[c[0] for c in CASES])
def test_nodal_solve_vs_oracle(name, n, boxes, per, mbe):
    """Same hierarchy, same cycle count, the max-norm residual before every
    cycle equal to 1e-6 (plus 1e-12 max|f| at the roundoff floor), solutions
    within 1e-9 rel-L2."""
    print(f"[nodal] solve {name}", flush=True)
    g, gphi, o, ophi, nl = _solve_pair(n, boxes, per, mbe)
    assert nl == o["nlevels"]
    assert g["converged"] and o["converged"]
    assert g["iters"] == o["iters"], (g["history"], o["history"])
    nf = o["normf"]
    for k, (a, b) in enumerate(zip(g["history"], o["history"])):
        assert abs(a - b) <= 1e-6 * b + 1e-12 * nf, (k, a, b)
    e = rel_l2(gphi, ophi)
    print(f"  {g['iters']} cycles, rel-L2 vs oracle {e:.2e}")
    assert e <= 1e-9


@pytest.mark.gpu
@pytest.mark.parametrize("name,n,boxes,per,mbe", CASES[:4], ids=[c[0] for c in CASES[:4]])
def test_nodal_one_cycle_elementwise(name, n, boxes, per, mbe):
    """After one V-cycle from zero the iterates agree node by node."""
    print(f"[nodal] one cycle {name}", flush=True)
    g, gphi, o, ophi, _ = _solve_pair(n, boxes, per, mbe, max_iter=1)
    assert g["iters"] == 1 and o["iters"] == 1
    assert np.abs(gphi - ophi).max() <= 1e-12 * np.abs(ophi).max()


@pytest.mark.gpu
def test_nodal_graph_replay_bitwise():
    P = lib()
    n, boxes, per = 64, W.uniform_boxes(64, 32), (False, True, False)
    sigma, f = _inputs(n, boxes, per)
    outs = []
    for graph in (1, 0):
        s = _gpu(n, boxes, per, sigma, dict(use_graph=graph, max_iter=4))
        rhs = _nodal_mf(P, boxes, f, n, per, 0)
        phi = s.node_mf(0, fill=0.0)
        s.solve(phi, rhs, 1e-10, raise_on_fail=False)
        torch.cuda.synchronize()
        outs.append(phi.to_numpy())
        s.close()
    assert all(np.array_equal(a, b) for a, b in zip(*outs))


@pytest.mark.gpu
def test_nodal_errors():
    P = lib()
    n, boxes = 16, W.uniform_boxes(16, 8)
    with pytest.raises(P.MGError):
        P.NodalMLMG(boxes, W.domain_box(n), (False,) * 3, opts=dict(precision=1))
    with pytest.raises(P.MGError):
        P.NodalMLMG(boxes, W.domain_box(n), (False,) * 3, opts=dict(nu1=0))
    with pytest.raises(P.MGError):  # cannot coarsen once
        P.NodalMLMG(boxes, W.domain_box(n), (False,) * 3, opts=dict(min_bottom_edge=16))
    with pytest.raises(P.MGError):  # boxes do not cover the domain
        P.NodalMLMG(boxes[:-1], W.domain_box(n), (False,) * 3)
    s = P.NodalMLMG(boxes, W.domain_box(n), (False,) * 3)
    cell = P.MultiFab(boxes, 0, fill=0.0)
    with pytest.raises(P.MGError) as ei:
        s.solve(s.node_mf(0, fill=0.0), cell)
    assert ei.value.code == P._lib.MG_ERR_MISMATCH
    # zero rhs: zero solution, converged without a cycle
    phi = s.node_mf(1, fill=5.0)
    info = s.solve(phi, s.node_mf(0, fill=0.0), history=True)
    assert info["converged"] and info["iters"] == 0
    got, _ = _unknowns(phi, boxes, n, (False,) * 3)
    assert np.all(got == 0.0)
    # non-convergence is reported with the iterate written
    sigma, f = _inputs(n, boxes, (False,) * 3)
    s2 = _gpu(n, boxes, (False,) * 3, sigma, dict(max_iter=2))
    info = s2.solve(s2.node_mf(0, fill=0.0), _nodal_mf(P, boxes, f, n, (False,) * 3, 0), 1e-14,
                    raise_on_fail=False)
    assert info["status"] == P._lib.MG_ERR_NOT_CONVERGED and info["iters"] == 2
    s.close()
    s2.close()


def _window_residual(sigma, per, G_phi, G_f, a, w):
    """max |f - A phi| over the nodes a+2 .. a+w-2 of the cell window a .. a+w-1,
    with the oracle's operator on that window (its boundary nodes read as 0,
    so only nodes whose 27 neighbours lie inside the window are kept)."""
    sl_c = tuple(slice(a[d], a[d] + w) for d in range(3))
    lev = ON.make_nodal_level(sigma[sl_c], (False,) * 3, h=(1.0 / sigma.shape[0],) * 3)
    sl_u = tuple(slice(a[d] + 1, a[d] + w) for d in range(3))
    Aphi = ON.apply_nodal(lev, G_phi[sl_u])
    r = G_f[sl_u] - Aphi
    return np.abs(r[1:-1, 1:-1, 1:-1]).max()


@pytest.mark.gpu
def test_nodal_full_size_256():
    """256^3 cells in 64 boxes of 64^3 (the benchmark's configuration): the GPU
    operator against the oracle's on windows of the random field, and the
    converged solution's residual recomputed by the oracle's operator on
    windows (interior, at walls and corners)."""
    print("[nodal] 256^3 full size", flush=True)
    P = lib()
    n = 256
    cfg = W.config_nodal(n, 64)
    boxes, per = cfg["boxes"], cfg["periodic"]
    sigma, f = cfg["sigma_cells"], cfg["rhs_unknowns"]
    s = _gpu(n, boxes, per, sigma, dict(min_bottom_edge=4))
    rng = np.random.default_rng(21)
    wins = [(0, 0, 0), (n - 20, n - 20, n - 20), (0, 100, n - 20)] + \
        [tuple(int(x) for x in rng.integers(0, n - 20, 3)) for _ in range(5)]
    # operator
    x = rng.standard_normal(W.nodal_unknown_shape(n, per))
    Gx = W.nodes_from_unknowns(x, n, per)
    out = s.node_mf(0)
    s.apply(P.MultiFab.from_numpy(boxes, W.scatter_nodes(Gx, boxes, 0), 0, ixtype=(1, 1, 1)), out)
    torch.cuda.synchronize()
    got, Gy = _unknowns(out, boxes, n, per)
    del got
    for a in wins:
        sl_c = tuple(slice(a[d], a[d] + 20) for d in range(3))
        lev = ON.make_nodal_level(sigma[sl_c], (False,) * 3, h=(1.0 / n,) * 3)
        sl_u = tuple(slice(a[d] + 1, a[d] + 20) for d in range(3))
        ref = ON.apply_nodal(lev, Gx[sl_u])[1:-1, 1:-1, 1:-1]
        g = Gy[sl_u][1:-1, 1:-1, 1:-1]
        assert np.abs(g - ref).max() <= 1e-13 * np.abs(ref).max(), a
    # solve
    rhs = _nodal_mf(P, boxes, f, n, per, 0)
    phi = s.node_mf(0, fill=0.0)
    info = s.solve(phi, rhs, 1e-10, history=True)
    torch.cuda.synchronize()
    assert info["converged"]
    h = info["history"]
    print(f"  {info['iters']} cycles, rel resid {info['rel_resid']:.2e}")
    _, Gp = _unknowns(phi, boxes, n, per)
    Gf = W.nodes_from_unknowns(f, n, per)
    normf = np.abs(f).max()
    for a in wins:
        r = _window_residual(sigma, per, Gp, Gf, a, 20)
        assert r <= 1e-10 * normf * 1.001 + 1e-13, (a, r / normf)
    assert h[-1] <= 1e-10 * normf and h[0] == pytest.approx(normf)
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("name,n,boxes,per,mbe", CASES, ids=[c[0] for c in CASES])
def test_nodal_pcg_vs_oracle(name, n, boxes, per, mbe):
    """CG preconditioned by one V-cycle per iteration: same iteration count,
    the recurrence residual's max norm equal to 1e-6 (plus the floor) at every
    iteration, solutions within 1e-9 rel-L2 of the oracle's."""
    print(f"[nodal] pcg {name}", flush=True)
    P = lib()
    sigma, f = _inputs(n, boxes, per)
    s = _gpu(n, boxes, per, sigma, dict(bottom_rel_tol=TIGHT, min_bottom_edge=mbe, krylov=1))
    rhs = _nodal_mf(P, boxes, f, n, per, 0)
    phi = s.node_mf(1, fill=0.0)
    g = s.solve(phi, rhs, 1e-10, history=True)
    torch.cuda.synchronize()
    got, _ = _unknowns(phi, boxes, n, per)
    ophi, o = ON.nodal_pcg_solve(sigma, per, f, 1e-10, opts=ON.NodalOpts(
        bottom_tol=TIGHT, min_bottom_cells=mbe))
    s.close()
    assert g["converged"] and o["converged"]
    assert g["iters"] == o["iters"], (g["history"], o["history"])
    nf = o["normf"]
    for k, (a, b) in enumerate(zip(g["history"], o["history"])):
        assert abs(a - b) <= 1e-6 * b + 1e-12 * nf, (k, a, b)
    e = rel_l2(got, ophi)
    print(f"  {g['iters']} iterations, rel-L2 vs oracle {e:.2e}")
    assert e <= 1e-9
    # the same solution as the V-cycle solve
    vphi, _ = ON.nodal_solve(sigma, per, f, 1e-12, opts=ON.NodalOpts(bottom_tol=TIGHT,
                                                                      min_bottom_cells=mbe))
    assert rel_l2(got, vphi) <= 1e-8


@pytest.mark.gpu
def test_nodal_pcg_full_size_256():
    """256^3 in the benchmark's configuration with the Krylov solve: the
    converged solution's residual recomputed by the oracle's operator on
    windows."""
    print("[nodal] pcg 256^3 full size", flush=True)
    P = lib()
    n = 256
    cfg = W.config_nodal(n, 64)
    boxes, per = cfg["boxes"], cfg["periodic"]
    sigma, f = cfg["sigma_cells"], cfg["rhs_unknowns"]
    s = _gpu(n, boxes, per, sigma, dict(min_bottom_edge=4, krylov=1))
    phi = s.node_mf(0, fill=0.0)
    info = s.solve(phi, _nodal_mf(P, boxes, f, n, per, 0), 1e-10)
    torch.cuda.synchronize()
    assert info["converged"]
    print(f"  {info['iters']} iterations, rel resid {info['rel_resid']:.2e}")
    _, Gp = _unknowns(phi, boxes, n, per)
    Gf = W.nodes_from_unknowns(f, n, per)
    normf = np.abs(f).max()
    rng = np.random.default_rng(22)
    wins = [(0, 0, 0), (n - 20, n - 20, n - 20)] + \
        [tuple(int(x) for x in rng.integers(0, n - 20, 3)) for _ in range(4)]
    for a in wins:
        r = _window_residual(sigma, per, Gp, Gf, a, 20)
        assert r <= 1e-10 * normf * 1.001 + 1e-13, (a, r / normf)
    s.close()
