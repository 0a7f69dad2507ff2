"""GPU parity of the float32 (differentiable) path.

Forward: the float32 distances are the unique fixed point of float32
relaxation, so they equal the float32-arithmetic oracle bit for bit, and
the canonical tree (pred, pred_edge) matches too; against the exact float64
oracle the relative error stays within 1e-5.  Backward: subtree sums of an
integer upstream gradient are exact integers, so they equal the oracle's;
the autograd Function reproduces them and agrees with float64 central
finite differences (h = 1e-2) on tree-stable edges.
"""
import sys

import numpy as np
import pytest
import torch

import graphgen as gg
import paper_1911_07260_amd as og

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def case(kind):
    if kind == "grid":
        g = gg.grid(64, 64, 1, 2, seed=0)
    elif kind == "road":
        g = gg.road(256, seed=2)
    else:
        g = gg.rmat(14, 16, seed=1)
    w = gg.float_weights(g, 1.0, 1000.0, seed=9)
    return g, w


@pytest.mark.parametrize("flags", [0, og.OG_FLAG_DEGREE_BINS])
@pytest.mark.parametrize("kind", ["grid", "road", "rmat"])
@pytest.mark.parametrize("delta,update", [(512, 1), (4096, 1), (512, 0), (1 << 16, 1)])
def test_forward_bit_exact_vs_f32_oracle(orc, kind, delta, update, flags):
    g, w = case(kind)
    dg = og.DeviceGraph.from_host(g, DEV)
    wt = torch.from_numpy(w).to(DEV)
    s = int(gg.pick_sources(g, 1, seed=4)[0])
    say(f"f32 forward {kind} delta={delta} update={update} flags={flags}")
    d, p, pe, st = og.sssp_f32(dg, wt, s, og.Schedule(delta=delta, update=update, flags=flags))
    torch.cuda.synchronize()
    d, p, pe = d.cpu().numpy(), p.cpu().numpy(), pe.cpu().numpy()
    ref = orc.dijkstra_real(g, w, s, f32=True)
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(d), fin)
    assert np.array_equal(d[fin], ref[fin].astype(np.float32))
    rp, rpe = orc.tree_real(g, w, s, ref, f32=True)
    assert np.array_equal(p, rp) and np.array_equal(pe, rpe)
    exact = orc.dijkstra_real(g, w, s, f32=False)
    nz = fin & (exact > 0)
    assert np.max(np.abs(d[nz] - exact[nz]) / exact[nz]) <= 1e-5


def test_backward_matches_oracle_subtree_sums(orc):
    g, w = case("road")
    dg = og.DeviceGraph.from_host(g, DEV)
    wt = torch.from_numpy(w).to(DEV)
    s = int(gg.pick_sources(g, 1, seed=5)[0])
    d, p, pe, _ = og.sssp_f32(dg, wt, s, og.Schedule(delta=1024))
    rng = np.random.default_rng(1)
    targets = rng.integers(0, g.n, size=1024)
    up = np.bincount(targets, minlength=g.n).astype(np.float32)
    say("backward, integer upstream")
    gw = og.sssp_backward_f32(dg, wt, p, pe, torch.from_numpy(up).to(DEV))
    torch.cuda.synchronize()
    ref_d = orc.dijkstra_real(g, w, s, f32=True)
    rp, rpe = orc.tree_real(g, w, s, ref_d, f32=True)
    up64 = np.where(np.isfinite(ref_d), up, 0).astype(np.float64)
    want = orc.subtree_grad(g, ref_d, rp, rpe, up64)
    assert np.array_equal(gw.cpu().numpy(), want.astype(np.float32))
    say("backward, real upstream")
    upr = rng.standard_normal(g.n).astype(np.float32)
    gw = og.sssp_backward_f32(dg, wt, p, pe, torch.from_numpy(upr).to(DEV)).cpu().numpy()
    want = orc.subtree_grad(g, ref_d, rp, rpe, np.where(np.isfinite(ref_d), upr, 0).astype(np.float64))
    assert np.allclose(gw, want, rtol=1e-5, atol=1e-3)


def test_autograd_and_finite_differences(orc):
    g = gg.road(48, seed=8)
    w = gg.float_weights(g, 1.0, 1000.0, seed=8)
    dg = og.DeviceGraph.from_host(g, DEV)
    s = int(gg.pick_sources(g, 1, seed=6)[0])
    rng = np.random.default_rng(2)
    targets = torch.from_numpy(rng.integers(0, g.n, size=64)).to(DEV)
    wt = torch.from_numpy(w).to(DEV).requires_grad_(True)
    say("autograd loss = sum of distances to 64 targets")
    dist = og.shortest_path_distances(wt, dg, s, og.Schedule(delta=512))
    reach = torch.isfinite(dist[targets])
    loss = dist[targets][reach].sum()
    loss.backward()
    grad = wt.grad.cpu().numpy().astype(np.float64)
    tg = targets[reach].cpu().numpy()
    h = 1e-2

    def L(wv):
        d = orc.dijkstra_real(g, wv, s, f32=False)
        return float(np.sum(d[tg]))

    checked = 0
    for e in rng.choice(g.m, size=150, replace=False):
        wp, wm = w.astype(np.float64).copy(), w.astype(np.float64).copy()
        wp[e] += h
        wm[e] -= h
        step = float(np.float32(wp[e]) - np.float32(wm[e]))
        fd = (L(wp.astype(np.float32)) - L(wm.astype(np.float32))) / step
        if abs(fd - round(fd)) < 1e-3:
            assert abs(fd - grad[e]) <= 1e-3 * max(1.0, abs(fd)), (e, fd, grad[e])
            checked += 1
    assert checked > 120


def test_invalid_weights():
    g = gg.from_edges(3, [0, 1], [1, 2], [1, 1])
    dg = og.DeviceGraph.from_host(g, DEV)
    for bad in (-1.0, float("nan"), float("inf")):
        wt = torch.tensor([1.0, bad], dtype=torch.float32, device=DEV)
        say(f"f32 bad weight {bad}")
        _, _, _, st = og.sssp_f32(dg, wt, 0, og.Schedule(delta=4), check=False)
        assert st["status"] == og.OG_ERR_NEGATIVE_WEIGHT


@pytest.mark.slow
def test_config_scale_road2048(orc):
    """Road-like 2048^2, float32 weights U(1,1000), 1,024 targets: forward
    bit-exact vs the float32 oracle, backward exact vs its subtree sums."""
    g = gg.road(2048, seed=0)
    w = gg.float_weights(g, 1.0, 1000.0, seed=3)
    dg = og.DeviceGraph.from_host(g, DEV)
    wt = torch.from_numpy(w).to(DEV)
    s = int(gg.pick_sources(g, 1, seed=1)[0])
    say("road2048 f32 forward + backward")
    d, p, pe, _ = og.sssp_f32(dg, wt, s, og.Schedule(delta=4096))
    targets = gg.pick_sources(g, 1024, seed=3)
    up = np.bincount(targets, minlength=g.n).astype(np.float32)
    gw = og.sssp_backward_f32(dg, wt, p, pe, torch.from_numpy(up).to(DEV))
    torch.cuda.synchronize()
    ref = orc.dijkstra_real(g, w, s, f32=True)
    fin = np.isfinite(ref)
    dn = d.cpu().numpy()
    assert np.array_equal(dn[fin], ref[fin].astype(np.float32)) and np.all(np.isinf(dn[~fin]))
    rp, rpe = orc.tree_real(g, w, s, ref, f32=True)
    want = orc.subtree_grad(g, ref, rp, rpe, np.where(fin, up, 0).astype(np.float64))
    assert np.array_equal(gw.cpu().numpy(), want.astype(np.float32))
