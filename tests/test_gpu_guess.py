"""GPU parity of the learned initial guess against the CPU oracle: pair list,
descriptors and frames, block rotation both ways, BF16 MFMA forward and
gradient (FP32 accumulation) against the FP64 network, Adam, and the guess
inside SCF (fallback and gain)."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import guess as G

pytestmark = pytest.mark.gpu

MODEL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_1708_00033_amd", "models", "guess_water.npy")


def _hfx():
    from paper_1708_00033_amd import hfx
    return hfx


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-30)


@pytest.fixture(scope="module")
def cluster():
    m = W.water_cluster(5, 61)
    ctx = _hfx().Context().load(m)
    counts = ctx.guess_setup()
    return m, ctx, counts


def test_pairs_features_frames(cluster):
    m, ctx, counts = cluster
    pairs = G.pair_list(m)
    X, P, R = ctx.guess_features()
    assert [tuple(p) for p in P] == [(a, b) for a, b, _ in pairs]
    assert tuple(np.bincount([t for _, _, t in pairs], minlength=3)) == counts
    Xo = G.features(m, pairs)
    assert np.abs(X - Xo).max() <= 1e-6 * max(1.0, np.abs(Xo).max())
    Ro = np.array([G.frame(m, a, b) for a, b, _ in pairs])
    assert np.abs(R - Ro).max() < 1e-12


def test_empty_environment_single_water():
    m = W.water_cluster(1, 3)
    ctx = _hfx().Context().load(m)
    counts = ctx.guess_setup()
    assert counts == (1, 2, 3)       # O self, two O-H, two H self + one H-H
    X, P, R = ctx.guess_features()
    pairs = G.pair_list(m)
    assert np.abs(X - G.features(m, pairs)).max() < 1e-6
    assert np.abs(R - np.array([G.frame(m, a, b) for a, b, _ in pairs])).max() < 1e-12


def test_block_rotation_both_ways(cluster):
    import torch
    m, ctx, counts = cluster
    pairs = G.pair_list(m)
    D = W.random_symmetric(m.nbf, 4, 0.3)
    Db = W.random_symmetric(m.nbf, 5, 0.3)
    dD, dDb = torch.tensor(D, device="cuda"), torch.tensor(Db, device="cuda")
    n = ctx.guess_packed_size()
    dT = torch.empty(n, dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    ctx.guess_targets_dev(dD.data_ptr(), dDb.data_ptr(), dT.data_ptr(), s)
    torch.cuda.synchronize()
    ref = np.concatenate([b.ravel() for b in G.local_blocks(m, pairs, D - Db)])
    assert ref.size == n
    assert np.abs(dT.cpu().numpy() - ref).max() <= 2e-7 * max(1.0, np.abs(ref).max())
    # assemble: FP32 blocks in, FP64 arithmetic on both sides
    blocks32 = np.random.default_rng(6).normal(size=n).astype(np.float32) * 0.05
    out = torch.empty_like(dD)
    ctx.guess_assemble_dev(torch.tensor(blocks32, device="cuda").data_ptr(), dDb.data_ptr(), out.data_ptr(), s)
    torch.cuda.synchronize()
    nb = G.block_sizes(m)
    split, o = [], 0
    for a, b, _ in pairs:
        k = nb[a] * nb[b]
        split.append(blocks32[o:o + k].astype(np.float64))
        o += k
    Do = G.assemble(m, pairs, split, Db)
    assert np.abs(out.cpu().numpy() - Do).max() < 1e-12
    assert np.abs(out.cpu().numpy() - out.cpu().numpy().T).max() < 1e-12


def _problem(ctx, m, counts, seed):
    rng = np.random.default_rng(seed)
    X, _, _ = ctx.guess_features()
    p = G.init_params(seed, fmean=X.mean(0), fscale=X.std(0) + 0.1, tscale=np.array([0.05, 0.03, 0.02]))
    for t, n in enumerate(G.HEAD_OUT):
        p[f"H{t}"] = rng.normal(size=(n, G.HIDDEN)) * 0.05
        p[f"c{t}"] = rng.normal(size=n) * 0.01
    T = [rng.normal(size=(c, n)) * 0.03 for c, n in zip(counts, G.HEAD_OUT)]
    flat = G.pack(p).astype(np.float32)
    return G.unpack(flat.astype(np.float64)), flat, X.astype(np.float64), T


def test_forward_and_gradient_match_fp64_network(cluster):
    import torch
    hfx = _hfx()
    m, ctx, counts = cluster
    p, flat, X, T = _problem(ctx, m, counts, 7)
    net = hfx.GuessNet(0, flat)
    dX = ctx.guess_features_dev()
    s = torch.cuda.current_stream().cuda_stream
    out = torch.empty(ctx.guess_packed_size(), dtype=torch.float32, device="cuda")
    net.forward_dev(dX, counts, out.data_ptr(), s)
    torch.cuda.synchronize()
    Y = out.cpu().numpy()
    ref = G.predict_blocks(p, X, counts)
    o = 0
    for t in range(3):
        k = counts[t] * G.HEAD_OUT[t]
        assert _rel(Y[o:o + k], ref[t]) < 2e-2, t
        o += k
    Tflat = torch.tensor(np.concatenate([x.ravel() for x in T]).astype(np.float32), device="cuda")
    loss = net.grad_dev(dX, counts, Tflat.data_ptr(), s)
    lo, go = G.loss_and_grad(p, X, counts, T)
    assert abs(loss - lo) <= 1e-2 * lo
    gr = G.unpack(net.get_grads().astype(np.float64))
    for name, _ in G.param_shapes()[:G.TRAINABLE]:
        assert _rel(gr[name], go[name]) < 2e-2, (name, _rel(gr[name], go[name]))
    for name, _ in G.param_shapes()[G.TRAINABLE:]:
        assert not gr[name].any()


def test_adam_matches_oracle(cluster):
    import torch
    hfx = _hfx()
    m, ctx, counts = cluster
    p, flat, X, T = _problem(ctx, m, counts, 8)
    net = hfx.GuessNet(0, flat)
    dX = ctx.guess_features_dev()
    s = torch.cuda.current_stream().cuda_stream
    Tflat = torch.tensor(np.concatenate([x.ravel() for x in T]).astype(np.float32), device="cuda")
    state = {}
    q = G.unpack(flat.astype(np.float64))
    for step in range(2):
        net.grad_dev(dX, counts, Tflat.data_ptr(), s)
        g = G.unpack(net.get_grads().astype(np.float64))
        net.adam(1e-3, s)
        G.adam(q, g, state, lr=1e-3)
        got = G.unpack(net.get_params().astype(np.float64))
        for name, _ in G.param_shapes():
            assert np.abs(got[name] - q[name]).max() < 2e-6, (step, name)


def test_gpu_training_reduces_loss(cluster):
    import torch
    hfx = _hfx()
    m, ctx, counts = cluster
    p, flat, X, T = _problem(ctx, m, counts, 9)
    net = hfx.GuessNet(0, flat)
    dX = ctx.guess_features_dev()
    s = torch.cuda.current_stream().cuda_stream
    Tflat = torch.tensor(np.concatenate([x.ravel() for x in T]).astype(np.float32), device="cuda")
    l0 = net.grad_dev(dX, counts, Tflat.data_ptr(), s)
    for _ in range(60):
        net.grad_dev(dX, counts, Tflat.data_ptr(), s, want_loss=False)
        net.adam(1e-3, s)
    l1 = net.grad_dev(dX, counts, Tflat.data_ptr(), s)
    assert l1 < 0.5 * l0, (l0, l1)


def test_untrained_network_is_sad_and_fallback():
    """Zero heads predict nothing: the learned start equals SAD.  A wildly
    scaled network fails the trace check and SCF falls back to SAD."""
    hfx = _hfx()
    m = W.water_cluster(3, 71)
    ctx = hfx.Context().load(m)
    p = G.init_params(1)
    for t in range(3):
        p[f"H{t}"][:] = 0.0
    zero = hfx.GuessNet(0, G.pack(p))
    r_sad = ctx.scf(e_tol=1e-10, d_rms_tol=1e-8)
    r_zero = ctx.scf(model=zero, e_tol=1e-10, d_rms_tol=1e-8)
    assert r_zero["guess_used"] == hfx.HFX_GUESS_LEARNED
    assert r_zero["iterations"] == r_sad["iterations"]
    assert abs(r_zero["energy"] - r_sad["energy"]) < 1e-9
    rng = np.random.default_rng(2)
    for t, n in enumerate(G.HEAD_OUT):
        p[f"H{t}"] = rng.normal(size=(n, G.HIDDEN))
    p["tscale"] = np.array([1e3, 1e3, 1e3])
    wild = hfx.GuessNet(0, G.pack(p))
    r_wild = ctx.scf(model=wild, e_tol=1e-10, d_rms_tol=1e-8)
    assert r_wild["guess_used"] == hfx.HFX_GUESS_SAD
    assert abs(r_wild["energy"] - r_sad["energy"]) < 1e-9


def test_trained_model_gains_over_sad():
    """The committed network (trained on converged densities of 4-32-water
    clusters) starts a held-out 32-water cluster closer to the converged
    density than SAD, needs no more SCF iterations, and reaches the same FP64
    energy."""
    import torch
    hfx = _hfx()
    assert os.path.exists(MODEL), "trained model missing"
    net = hfx.GuessNet(0, np.load(MODEL))
    m = W.water_cluster(32, 29_999)
    ctx = hfx.Context().load(m)
    r_sad = ctx.scf()
    r_nn = ctx.scf(model=net)
    assert r_sad["converged"] and r_nn["converged"]
    assert r_nn["guess_used"] == hfx.HFX_GUESS_LEARNED
    assert abs(r_nn["energy"] - r_sad["energy"]) < 1e-8
    assert r_nn["iterations"] <= r_sad["iterations"], (r_nn["iterations"], r_sad["iterations"])
    D_sad = ctx.sad_density()
    dD = torch.tensor(D_sad, device="cuda")
    assert ctx.guess_apply(net, dD.data_ptr(), torch.cuda.current_stream().cuda_stream)
    D_nn = dD.cpu().numpy()
    err_sad = np.linalg.norm(D_sad - r_sad["D"])
    err_nn = np.linalg.norm(D_nn - r_sad["D"])
    assert err_nn < 0.7 * err_sad, (err_nn, err_sad)
