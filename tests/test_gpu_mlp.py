"""The ODE surrogate on the GPU, through the C ABI, against the oracle.

Tolerances (bfloat16 operands, FP32 accumulation), derived from the
arithmetic:

* forward vs the oracle's quantised forward (bf16 weights and activations,
  FP64 accumulation): the two differ only by accumulation order (~1e-6
  relative) and the rare bf16 rounding flip of a hidden activation that this
  moves across a rounding boundary, so max |dy| <= 5e-3 and RMS <= 5e-4 on
  outputs of unit scale;
* forward vs the exact FP64 forward: quantisation error itself, RMS <= 2e-2
  relative to the output RMS (a handful of 2^-9 roundings per path);
* gradient vs the exact FP64 backward: normwise relative error <= 3e-2 per
  parameter block (weights, activations and back-propagated errors each
  rounded to bf16: ~sqrt(6) x 2^-9 ~ 5e-3 expected, 6x margin), loss within
  1e-2 relative.
A wrong operand order, packing permutation, missing GELU' factor or bias
gives O(1) errors and fails every one of these.
"""
import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from oracle import ode as oode
from oracle.constants import DEFAULT as OP
from paper_2105_00448_amd import hca, synth

from mlp_bounds import host_net, quantised_forward_bound

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def blocks(theta):
    out, o = {}, 0
    for name, shape in omlp.SHAPES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n]
        o += n
    return out


def random_theta(seed):
    rng = np.random.default_rng(seed)
    t = omlp.init_params(seed)
    p = omlp.unpack(t)
    for k in p:   # nonzero biases so that their path is exercised
        if k.startswith("b"):
            p[k] = 0.3 * rng.standard_normal(p[k].shape)
    return omlp.pack(p).astype(np.float32)


def trainer_on(X, Y, seed=0):
    Xd = torch.tensor(X, dtype=torch.float32, device=DEV)
    Yd = torch.tensor(Y, dtype=torch.float32, device=DEV)
    return hca.Trainer(Xd, Yd, seed=seed), Xd, Yd


@pytest.mark.parametrize("n", [1, 63, 64, 1000, 4133])
def test_forward_matches_quantised_oracle(n):
    print(f"\n[mlp forward] n={n}", flush=True)
    rng = np.random.default_rng(n)
    X = rng.standard_normal((max(n, 2), 6)).astype(np.float32)
    Y = rng.standard_normal((max(n, 2), 3)).astype(np.float32)
    tr, Xd, _ = trainer_on(X, Y)
    theta = random_theta(7)
    tr.set_params(theta)
    Xs = torch.tensor(X[:n], device=DEV)
    out = torch.empty((n, 3), dtype=torch.float32, device=DEV)
    tr.eval(Xs, out, raw=False)
    got = out.cpu().numpy().astype(np.float64)
    th64 = theta.astype(np.float64)
    ref_q = omlp.quantised_forward(th64, X[:n].astype(np.float64))
    d = np.abs(got - ref_q)
    assert d.max() <= 5e-3, d.max()
    assert np.sqrt((d ** 2).mean()) <= 5e-4
    ref = omlp.forward(th64, X[:n].astype(np.float64))
    rms = np.sqrt((ref ** 2).mean())
    assert np.sqrt(((got - ref) ** 2).mean()) <= 2e-2 * rms
    tr.close()


def test_statistics_and_standardisation():
    rng = np.random.default_rng(11)
    n = 20000
    X = (rng.standard_normal((n, 6)) * [3, 0.1, 0, 1e-3, 2e-3, 0.3] + [15, 0.5, 0, 0.02, 0.2, 0.5])
    Y = rng.standard_normal((n, 3)) * [1e-5, 1e-4, 1e-3] + [1e-5, 0, 2e-3]
    X = X.astype(np.float32)
    Y = Y.astype(np.float32)
    tr, _, _ = trainer_on(X, Y)
    st = tr.export().stats()
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
    np.testing.assert_allclose(st["in_mean"], X64.mean(0), rtol=1e-5, atol=1e-9)
    sd = X64.std(0)
    scale = np.where(sd > 0, 1.0 / np.where(sd > 0, sd, 1), 1.0)   # zero-spread column: scale 1
    np.testing.assert_allclose(st["in_scale"], scale, rtol=1e-4)
    np.testing.assert_allclose(st["out_mean"], Y64.mean(0), rtol=1e-5, atol=1e-12)
    np.testing.assert_allclose(st["out_scale"], Y64.std(0), rtol=1e-4)
    np.testing.assert_array_equal(st["in_lo"], X.min(0))
    np.testing.assert_array_equal(st["in_hi"], X.max(0))
    Xs = torch.empty((n, 6), device=DEV)
    Ys = torch.empty((n, 3), device=DEV)
    tr.data(Xs, Ys)
    np.testing.assert_allclose(Xs.cpu().numpy(), (X64 - st["in_mean"]) * st["in_scale"], rtol=1e-5,
                               atol=1e-5)
    np.testing.assert_allclose(Ys.cpu().numpy(), (Y64 - st["out_mean"]) / st["out_scale"], rtol=1e-5,
                               atol=1e-5)
    tr.close()


@pytest.mark.parametrize("batch", [64, 256, 1024])
def test_gradient_matches_oracle(batch):
    print(f"\n[mlp gradient] batch={batch}", flush=True)
    rng = np.random.default_rng(batch)
    n = 5000
    X = (rng.standard_normal((n, 6)) * 2 + 1).astype(np.float32)
    Xr = X.astype(np.float64)
    Y = np.stack([np.sin(Xr[:, 0]), Xr[:, 1] * Xr[:, 2], np.tanh(Xr[:, 3] - Xr[:, 5])], 1)
    Y = Y.astype(np.float32)
    tr, _, _ = trainer_on(X, Y)
    theta = random_theta(3)
    tr.set_params(theta)
    Xs = torch.empty((n, 6), device=DEV)
    Ys = torch.empty((n, 3), device=DEV)
    tr.data(Xs, Ys)
    idx = rng.integers(0, n, batch).astype(np.int32)
    g = torch.empty(hca.MLP_NPARAM, dtype=torch.float32, device=DEV)
    loss = tr.gradient(torch.tensor(idx, device=DEV), g)
    Xb = Xs.cpu().numpy().astype(np.float64)[idx]
    Yb = Ys.cpu().numpy().astype(np.float64)[idx]
    L, gref = omlp.backward(theta.astype(np.float64), Xb, Yb)
    assert abs(loss - L) <= 1e-2 * L
    got = blocks(g.cpu().numpy().astype(np.float64))
    ref = blocks(gref)
    for name in got:
        err = np.linalg.norm(got[name] - ref[name]) / np.linalg.norm(ref[name])
        assert err <= 3e-2, (name, err)
    tr.close()


def test_gradient_is_batch_additive():
    """The gradient of a batch is the sum of its 64-sample workgroup parts
    (fixed-order reduction): two halves add up to the whole."""
    rng = np.random.default_rng(5)
    n = 3000
    X = rng.standard_normal((n, 6)).astype(np.float32)
    Y = rng.standard_normal((n, 3)).astype(np.float32)
    tr, _, _ = trainer_on(X, Y)
    tr.set_params(random_theta(9))
    idx = torch.tensor(rng.integers(0, n, 256).astype(np.int32), device=DEV)
    g = torch.empty(hca.MLP_NPARAM, device=DEV)
    g1 = torch.empty_like(g)
    g2 = torch.empty_like(g)
    tr.gradient(idx, g)
    tr.gradient(idx[:128].contiguous(), g1)
    tr.gradient(idx[128:].contiguous(), g2)
    # halves are normalised by 128, the whole by 256
    np.testing.assert_allclose(g.cpu().numpy(), 0.5 * (g1 + g2).cpu().numpy(), rtol=1e-4, atol=1e-7)
    tr.close()


def test_gradient_rejects_bad_batch():
    X = np.zeros((100, 6), np.float32)
    Y = np.zeros((100, 3), np.float32)
    tr, _, _ = trainer_on(X, Y)
    g = torch.empty(hca.MLP_NPARAM, device=DEV)
    idx = torch.zeros(128, dtype=torch.int32, device=DEV)
    for b in (0, 63, 100):
        st = tr._lib.hca_mlp_gradient(tr._h, idx.data_ptr(), b, g.data_ptr(), None)
        assert st == hca.E_RANGE, (b, st)
    with pytest.raises(hca.HcaError):
        tr.train(1, batch=96)
    tr.close()


# ---- harvest, training and the surrogate in the coupled step -----------------------

@pytest.fixture(scope="module")
def harvested():
    """Training pairs from the plain integrator: 32^3 lattices (8 Gaussians),
    three seeds, bolus of both drugs at step 0, 12 coupled steps each."""
    print("\n[harvest] 3 seeds x 12 steps on 32^3", flush=True)
    Xs, Ys = [], []
    for seed in (1, 2, 3):
        tis = synth.make_tissue(32, 8, seed=seed)
        sched = synth.bolus_schedule([0])
        with hca.Simulation([(tis.cell, tis.w, tis.seed, (sched.times, sched.amts))]) as sim:
            cap = tis.cell.size
            X = torch.empty((cap, 6), device=DEV)
            Y = torch.empty((cap, 3), device=DEV)
            for _ in range(12):
                n = sim.harvest_step(X, Y)
                Xs.append(X[:n].clone())
                Ys.append(Y[:n].clone())
    return torch.cat(Xs), torch.cat(Ys)


def test_harvest_rows_are_the_plain_step():
    tis = synth.make_tissue(24, 6, seed=4)
    sched = synth.bolus_schedule([0])
    rep = (tis.cell, tis.w, tis.seed, (sched.times, sched.amts))
    with hca.Simulation([rep]) as a, hca.Simulation([rep]) as b:
        a.step(2)
        b.step(2)
        before = {k: b.field(k) for k in ("L", "P", "Vc", "phi")}
        cap = tis.cell.size
        X = torch.empty((cap, 6), device=DEV)
        Y = torch.empty((cap, 3), device=DEV)
        n = a.harvest_step(X, Y)
        b.run_phases(hca.PH_O2 | hca.PH_DRUGS)
        mid = {k: b.field(k) for k in ("K", "G1", "G2")}
        b.run_phases(hca.PH_ODE)
        after = {k: b.field(k) for k in ("P", "Vc", "phi")}
        b.run_phases(hca.PH_CA | hca.PH_STATS | hca.PH_ADVANCE)
        occ = before["L"].ravel() != 0
        assert n == occ.sum()
        Xh = X[:n].cpu().numpy()
        Yh = Y[:n].cpu().numpy()
        exp_x = np.stack([mid["K"].ravel(), mid["G1"].ravel(), mid["G2"].ravel(),
                          before["P"].ravel(), before["Vc"].ravel(), before["phi"].ravel()], 1)[occ]
        np.testing.assert_array_equal(Xh, exp_x.astype(np.float32))
        np.testing.assert_array_equal(Yh[:, 0], (after["P"].ravel() - before["P"].ravel())[occ]
                                      .astype(np.float32))
        np.testing.assert_array_equal(Yh[:, 1], (after["Vc"].ravel() - before["Vc"].ravel())[occ]
                                      .astype(np.float32))
        cancer = before["L"].ravel()[occ] == 1
        dphi = (after["phi"].ravel() - before["phi"].ravel())[occ][cancer]
        np.testing.assert_allclose(Yh[cancer, 2], dphi, rtol=1e-6)
        # the harvest step is an ordinary plain step
        for k in ("L", "K", "G1", "G2", "P", "Vc", "phi"):
            np.testing.assert_array_equal(a.field(k), b.field(k))
        # cap too small: range error before any work
        with pytest.raises(hca.HcaError) as e:
            a.harvest_step(X[: n // 2], Y[: n // 2])
        assert e.value.status == hca.E_RANGE
        assert a.stats()["step"] == 3


@pytest.fixture(scope="module")
def trained(harvested):
    X, Y = harvested
    print(f"\n[train] {X.shape[0]} pairs", flush=True)
    tr = hca.Trainer(X, Y, seed=1)
    losses = tr.train(1500, batch=1024, lr=2e-3)
    losses2 = tr.train(1500, batch=1024, lr=5e-4)
    yield tr, np.concatenate([losses, losses2])
    tr.close()


def test_training_reduces_loss(trained):
    tr, losses = trained
    first = losses[:20].mean()
    last = losses[-100:].mean()
    print(f"\n[train] loss {first:.3e} -> {last:.3e}", flush=True)
    assert np.all(np.isfinite(losses))
    assert last < 0.02 * first


def test_surrogate_step_follows_the_rule(trained):
    """ODE phase with the surrogate: voxels whose predicted phi lands within
    the margin of 1 are exactly the plain integrator's; all others take the
    network's update (checked against the network evaluated on the same
    inputs); counts add up."""
    tr, _ = trained
    net = tr.export()
    margin = 1e-3
    tis = synth.make_tissue(32, 8, seed=9)   # a seed not in the training set
    sched = synth.bolus_schedule([0])
    rep = (tis.cell, tis.w, tis.seed, (sched.times, sched.amts))
    with hca.Simulation([rep]) as s, hca.Simulation([rep]) as p:
        for sim in (s, p):
            sim.step(3)
            sim.run_phases(hca.PH_O2 | hca.PH_DRUGS)
        s.set_surrogate(net, margin)
        L = s.field("L").ravel()
        occ = L != 0
        inp = np.stack([s.field(k).ravel() for k in ("K", "G1", "G2", "P", "Vc", "phi")], 1)[occ]
        Xd = torch.tensor(inp.astype(np.float32), device=DEV)
        pred = torch.empty((Xd.shape[0], 3), device=DEV)
        tr.eval(Xd, pred, raw=True)
        pred = pred.cpu().numpy().astype(np.float64)
        s.run_phases(hca.PH_ODE)
        p.run_phases(hca.PH_ODE)
        st = s.stats()
        assert st["sur_voxels"] + st["sur_fallbacks"] == occ.sum()
        got = {k: s.field(k).ravel()[occ] for k in ("P", "Vc", "phi")}
        plain = {k: p.field(k).ravel()[occ] for k in ("P", "Vc", "phi")}
        cancer = L[occ] == 1
        gap = np.abs(inp[:, 5] + pred[:, 2] - 1.0)
        fb = cancer & (gap < margin)
        sure = np.abs(gap - margin) > 1e-6          # decision not at the rounding edge
        assert fb[sure].sum() <= st["sur_fallbacks"] <= fb.sum() + (~sure).sum()
        for k, j in (("P", 0), ("Vc", 1)):
            m = fb & sure
            np.testing.assert_array_equal(got[k][m], plain[k][m])
            m = ~fb & sure
            np.testing.assert_allclose(got[k][m], inp[m, 3 + j] + pred[m, j], rtol=1e-6,
                                       atol=1e-6 * np.abs(pred[:, j]).max())
        m = fb & sure
        np.testing.assert_array_equal(got["phi"][m], plain["phi"][m])
        m = ~fb & sure & cancer
        np.testing.assert_allclose(got["phi"][m], inp[m, 5] + pred[m, 2], rtol=1e-6, atol=1e-9)
        m = ~cancer
        np.testing.assert_array_equal(got["phi"][m], inp[m, 5])   # stroma carries no clock


def surrogate_error(trained_net, seed, steps, margin=1e-3):
    """Run plain and surrogate side by side from one state for `steps` ODE
    phases on identical inputs (the plain state is copied into the surrogate
    context before each phase): per-step relative errors and decision flips."""
    tis = synth.make_tissue(32, 8, seed=seed)
    sched = synth.bolus_schedule([0])
    rep = (tis.cell, tis.w, tis.seed, (sched.times, sched.amts))
    out = []
    with hca.Simulation([rep]) as s, hca.Simulation([rep]) as p:
        s.set_surrogate(trained_net, margin)
        for _ in range(steps):
            p.run_phases(hca.PH_O2 | hca.PH_DRUGS)
            for k in ("L", "K", "G1", "G2", "P", "Vc", "phi"):
                s.set_field(k, p.field(k))
            p.run_phases(hca.PH_ODE)
            s.run_phases(hca.PH_ODE)
            L = p.field("L")
            occ = L != 0
            can = L == 1
            e = {}
            for k in ("P", "Vc"):
                a, b = s.field(k)[occ], p.field(k)[occ]
                e[k] = np.abs(a - b).max() / np.abs(b).max()
            a, b = s.field("phi")[can], p.field("phi")[can]
            e["phi"] = np.abs(a - b).max() / np.abs(b).max()
            e["flips"] = int(np.count_nonzero((a >= 1.0) != (b >= 1.0)))
            e["cancer"] = int(can.sum())
            out.append(e)
            p.run_phases(hca.PH_CA | hca.PH_STATS | hca.PH_ADVANCE)
    return out


def test_surrogate_error_and_flip_rate(trained):
    tr, _ = trained
    errs = surrogate_error(tr.export(), seed=9, steps=6)
    for e in errs:
        print(f"\n[surrogate error] {e}", flush=True)
        assert e["P"] <= 1e-2 and e["Vc"] <= 1e-2 and e["phi"] <= 1e-2
        # the margin sends every cell near the threshold to the plain integrator
        assert e["flips"] == 0


# ---- Adam, the gradient element by element, the in-step apply kernel ---------------

def adam_error_bound(theta0, grads, lr, b1, b2, eps):
    """The oracle's Adam trajectory in FP64 from theta0 over the gradients,
    and a running bound on the error of the same steps in FP32: the moments
    m = b1 m + (1 - b1) g and v = b2 v + (1 - b2) g^2 carry their previous
    error (times b1, b2) plus a few roundings of their terms' magnitudes;
    the update lr m bc1 / (sqrt(v bc2) + eps) (bias corrections bc rounded
    once) inherits the moments' errors through its derivatives plus about
    eight roundings; theta -= update adds one rounding of theta."""
    u = 2.0 ** -24
    th = theta0.astype(np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    Em = np.zeros_like(th)
    Ev = np.zeros_like(th)
    Eth = np.zeros_like(th)
    for k, g in enumerate(grads, 1):
        g = g.astype(np.float64)
        Em = b1 * Em + 3 * u * (np.abs(b1 * m) + np.abs((1 - b1) * g))
        Ev = b2 * Ev + 4 * u * (np.abs(b2 * v) + np.abs((1 - b2) * g * g))
        th_new, m, v = omlp.adam_step(th, m, v, g, k, lr, b1=b1, b2=b2, eps=eps)
        bc1 = 1.0 / (1.0 - b1 ** k)
        bc2 = 1.0 / (1.0 - b2 ** k)
        S = np.sqrt(v * bc2)
        rel_v = np.where(v > 0, Ev / np.where(v > 0, v, 1.0), 0.0)
        dS = 0.5 * S * rel_v + 2 * u * S + 0.5 * np.sqrt(Ev * bc2)
        upd = lr * m * bc1 / (S + eps)
        Eth = (Eth + lr * bc1 * Em / (S + eps) + np.abs(upd) * dS / (S + eps) + 8 * u * np.abs(upd)
               + u * np.abs(th_new))
        th = th_new
    return th, Eth


def test_adam_matches_oracle():
    """Four Adam steps of the library (FP32) from fixed parameters and fixed
    gradients (many decades, exact zeros, signs changing between steps)
    against the oracle's adam_step in FP64, element by element, within twice
    the running FP32 error bound of adam_error_bound.  The oracle takes the
    kernel's own constants (b1, b2, eps, lr as float32 values).  An
    emulation of the kernel's roundings stayed below 0.12 of the bound; a
    wrong moment, bias correction or step count is off by O(lr)."""
    rng = np.random.default_rng(21)
    X = rng.standard_normal((256, 6)).astype(np.float32)
    Y = rng.standard_normal((256, 3)).astype(np.float32)
    tr, _, _ = trainer_on(X, Y)
    theta0 = random_theta(4)
    tr.set_params(theta0)
    f32 = lambda x: float(np.float32(x))
    lr, b1, b2, eps = f32(2e-3), f32(0.9), f32(0.999), f32(1e-8)
    grads = []
    for k in range(4):
        g = rng.standard_normal(hca.MLP_NPARAM) * 10.0 ** rng.uniform(-6, 1, hca.MLP_NPARAM)
        g[rng.random(hca.MLP_NPARAM) < 0.02] = 0.0
        grads.append(g.astype(np.float32))
    for k, g in enumerate(grads):
        if k == 1:   # once from a device tensor
            tr.apply_gradient(torch.tensor(g, device=DEV), lr)
        else:
            tr.apply_gradient(g, lr)
        if k == 2:   # after three steps, and again after the fourth (t = 4)
            ref, E = adam_error_bound(theta0, grads[:3], lr, b1, b2, eps)
            err = np.abs(tr.params().astype(np.float64) - ref)
            assert np.all(err <= 2 * E), (err / (2 * E)).max()
    ref, E = adam_error_bound(theta0, grads, lr, b1, b2, eps)
    got = tr.params().astype(np.float64)
    err = np.abs(got - ref)
    print(f"\n[adam] max err/bound {(err / (2 * E)).max():.3f}", flush=True)
    assert np.all(err <= 2 * E), (err / (2 * E)).max()
    # the parameters did move (by about lr per step where the gradient is not 0)
    assert np.abs(got - theta0).max() > 2 * lr
    with pytest.raises(hca.HcaError):
        tr.apply_gradient(grads[0], -1.0)
    tr.close()


def abs_term_sums(theta, X, Y):
    """Per gradient element, the sum over the batch of the magnitudes of the
    products it adds up, |dZ| |H| (|dZ| for a bias), with the bfloat16
    operands of oracle.mlp.quantised_backward."""
    q = omlp.bf16
    p = omlp.unpack(theta)
    B = X.shape[0]
    W = {k: q(v) for k, v in p.items() if k.startswith("W")}
    h = [q(X)]
    z = []
    for i in (1, 2, 3):
        z.append(h[-1] @ W[f"W{i}"].T + p[f"b{i}"])
        h.append(q(omlp.gelu(z[-1])))
    y = h[3] @ W["W4"].T + p["b4"]
    dz = q(2.0 * (y - Y) / (B * omlp.NOUT))
    A = {"W4": np.abs(dz).T @ np.abs(h[3]), "b4": np.abs(dz).sum(0)}
    for i in (3, 2, 1):
        dz = q((dz @ W[f"W{i + 1}"]) * omlp.gelu_grad(z[i - 1]))
        A[f"W{i}"] = np.abs(dz).T @ np.abs(h[i - 1])
        A[f"b{i}"] = np.abs(dz).sum(0)
    return omlp.pack(A)


@pytest.mark.parametrize("batch", [64, 1024])
def test_gradient_elementwise_matches_quantised_oracle(batch):
    """The library's gradient against the oracle's gradient of the network
    with bfloat16 operands (oracle.mlp.quantised_backward), element by
    element.  The two differ by the kernel's FP32 accumulation (relative
    2^-24 per addition) and its tabulated forward GELU (error <= 8e-6 |z|);
    both can move an FP32 value across a bfloat16 rounding boundary, which
    changes that one operand by one bfloat16 step (at most 2^-7 of it).  A
    gradient element is a sum of products whose magnitudes add up to A_i,
    so the bar is |g_i - g_i,ref| <= 2^-7 A_i (an emulation of the kernel's
    rounding points stayed below 0.6 of it).  A wrong operand, packing slot,
    transposition, missing GELU' factor or bias term moves an element by
    O(|g_i|) ~ A_i/4.  Also normwise against the exact FP64 backward, the
    bfloat16 quantisation itself: <= 3e-2 per block."""
    print(f"\n[mlp gradient elementwise] batch={batch}", flush=True)
    rng = np.random.default_rng(100 + batch)
    n = 4000
    X = (rng.standard_normal((n, 6)) * 2 + 1).astype(np.float32)
    Xr = X.astype(np.float64)
    Y = np.stack([np.sin(Xr[:, 0]), Xr[:, 1] * Xr[:, 2], np.tanh(Xr[:, 3] - Xr[:, 5])], 1)
    tr, _, _ = trainer_on(X, Y.astype(np.float32))
    theta = random_theta(13)
    tr.set_params(theta)
    Xs = torch.empty((n, 6), device=DEV)
    Ys = torch.empty((n, 3), device=DEV)
    tr.data(Xs, Ys)
    idx = rng.integers(0, n, batch).astype(np.int32)
    g = torch.empty(hca.MLP_NPARAM, dtype=torch.float32, device=DEV)
    loss = tr.gradient(torch.tensor(idx, device=DEV), g)
    Xb = Xs.cpu().numpy().astype(np.float64)[idx]
    Yb = Ys.cpu().numpy().astype(np.float64)[idx]
    th = theta.astype(np.float64)
    Lq, gq = omlp.quantised_backward(th, Xb, Yb)
    A = abs_term_sums(th, Xb, Yb)
    got = g.cpu().numpy().astype(np.float64)
    ratio = np.abs(got - gq) / (2.0 ** -7 * A + 1e-30)
    worst = int(np.argmax(ratio))
    print(f"[mlp gradient elementwise] max |dg|/(2^-7 A) {ratio.max():.3f}, median "
          f"{np.median(ratio):.2e}; A/|g| median {np.median(A / (np.abs(gq) + 1e-30)):.2f}",
          flush=True)
    assert ratio.max() <= 1.0, (worst, got[worst], gq[worst], A[worst])
    assert abs(loss - Lq) <= 1e-3 * Lq
    _, gx = omlp.backward(th, Xb, Yb)
    for name, blk in blocks(got).items():
        ref = blocks(gx)[name]
        assert np.linalg.norm(blk - ref) <= 3e-2 * np.linalg.norm(ref), name
    tr.close()


def test_surrogate_apply_matches_oracle(case_sur):
    """The ODE phase with a surrogate set, on an oracle state, against the
    oracle: a voxel advanced by the network equals input + the oracle's
    quantised forward of the standardised input (bfloat16 operands) within
    that voxel's bound from quantised_forward_bound (plus the FP32 and FP64
    roundings of un-standardising and adding); a voxel sent to the plain
    integrator equals the oracle's ode_step (P, V_c <= 1e-10, phi
    bit-exact); empty voxels and stroma clocks are untouched.  The network
    is the oracle's initial parameters with random biases, its statistics
    computed here from the inputs, so every input comes from the oracle
    side.  A margin of 0.02 around phi = 1 sends a few hundred cells to the
    plain integrator; a voxel whose bound reaches across that edge may go
    either way and must match one of the two results."""
    tis, sched, s, theta, stats = case_sur
    margin = 0.02
    net, th32 = host_net(theta, stats)
    with hca.Simulation([(tis.cell, tis.w, tis.seed, (sched.times, sched.amts))],
                        hca.default_params()) as sim:
        for name in ("L", "K", "G1", "G2", "P", "Vc", "phi"):
            sim.set_field(name, getattr(s, name))
        sim.set_surrogate(net, margin)
        sim.run_phases(hca.PH_ODE)
        got = {k: sim.field(k).ravel() for k in ("P", "Vc", "phi")}
        st = sim.stats()
    L = s.L.ravel()
    occ = L != 0
    cancer = L == 1
    raw = np.stack([getattr(s, k).ravel() for k in ("K", "G1", "G2", "P", "Vc", "phi")], 1)
    # the kernel's FP32 standardisation, done identically in float32 here
    xs = (raw.astype(np.float32) - stats["in_mean"]) * stats["in_scale"]
    y, Ey = quantised_forward_bound(theta.astype(np.float64), xs[occ].astype(np.float64))
    sc = stats["out_scale"].astype(np.float64)
    mu = stats["out_mean"].astype(np.float64)
    upd = np.zeros((L.size, 3))
    upd[occ] = y * sc + mu
    tol = np.zeros((L.size, 3))
    base = np.stack([s.P.ravel(), s.Vc.ravel(), s.phi.ravel()], 1)
    tol[occ] = (Ey * sc + 2.0 ** -22 * (np.abs(y * sc) + np.abs(mu))
                + 2.0 ** -51 * (np.abs(base[occ]) + np.abs(upd[occ])))
    print(f"\n[surrogate apply] bound (standardised units): median "
          f"{np.median(Ey, axis=0)}, max {Ey.max(axis=0)}", flush=True)
    assert np.median(Ey) <= 2e-2        # informative: an O(1) error cannot hide
    Pp, Vp, php = oode.ode_step(s.L, s.K, s.P, s.Vc, s.phi, OP)
    Pp, Vp, php = Pp.ravel(), Vp.ravel(), php.ravel()
    gap = np.abs(s.phi.ravel() + upd[:, 2] - 1.0)
    edge = np.abs(gap - margin) <= tol[:, 2] + 1e-12
    fb_sure = cancer & (gap < margin) & ~edge
    net_sure = occ & ~fb_sure & ~(cancer & edge)
    undecided = cancer & edge
    assert fb_sure.sum() > 50 and net_sure.sum() > 5000
    # counts
    assert st["sur_voxels"] + st["sur_fallbacks"] == occ.sum()
    assert fb_sure.sum() <= st["sur_fallbacks"] <= fb_sure.sum() + undecided.sum()
    # plain-integrator voxels: the oracle's ODE step
    scaleP, scaleV = np.abs(Pp[occ]).max(), np.abs(Vp[occ]).max()
    assert np.abs(got["P"][fb_sure] - Pp[fb_sure]).max() <= 1e-10 * scaleP
    assert np.abs(got["Vc"][fb_sure] - Vp[fb_sure]).max() <= 1e-10 * scaleV
    assert np.array_equal(got["phi"][fb_sure], php[fb_sure])
    # network voxels: input + the quantised forward within the per-voxel bound
    for k, j in (("P", 0), ("Vc", 1), ("phi", 2)):
        m = net_sure & cancer if k == "phi" else net_sure
        dev = np.abs((got[k] - base[:, j]) - upd[:, j])[m]
        ratio = dev / tol[m, j]
        print(f"[surrogate apply] {k}: max |dev|/bound {ratio.max():.3f}, max |dev| in "
              f"standardised units {(dev / sc[j]).max():.2e}", flush=True)
        assert ratio.max() <= 1.0, k
    # stroma carries no clock; empty voxels are untouched
    stroma = L == 2
    assert np.array_equal(got["phi"][stroma], s.phi.ravel()[stroma])
    for k in ("P", "Vc", "phi"):
        assert np.array_equal(got[k][~occ], getattr(s, k).ravel()[~occ])
    # the undecided voxels took one of the two results
    for i in np.flatnonzero(undecided):
        plain = (abs(got["P"][i] - Pp[i]) <= 1e-10 * scaleP and got["phi"][i] == php[i])
        netw = abs((got["P"][i] - base[i, 0]) - upd[i, 0]) <= tol[i, 0]
        assert plain or netw, i


@pytest.mark.parametrize("precision", [64, 32])
def test_surrogate_apply_on_a_tiled_lattice_is_the_tiled_result(case_sur, precision):
    """Each voxel's surrogate update depends on that voxel alone (its own
    MFMA column; the plain integrator for fallbacks), so the ODE phase on
    the 32^3 state tiled 72 times along x (2.36 M voxels: work items of
    1152 voxels, each listed in two runs, the fallback list spanning both)
    is the 32^3 result tiled, bit for bit, with 72 times the counts."""
    tis, sched, s, theta, stats = case_sur
    margin = 0.02
    net, th32 = host_net(theta, stats)
    reps = 72
    names = ("L", "K", "G1", "G2", "P", "Vc", "phi")
    params = hca.default_params(precision=precision)

    def run(tile):
        cell = np.tile(tis.cell, (1, 1, tile))
        w = np.tile(tis.w, (1, 1, tile))
        with hca.Simulation([(cell, w, tis.seed, (sched.times, sched.amts))], params) as sim:
            for name in names:
                sim.set_field(name, np.tile(getattr(s, name), (1, 1, tile)))
            sim.set_surrogate(net, margin)
            sim.run_phases(hca.PH_ODE)
            return {k: sim.field(k) for k in ("P", "Vc", "phi")}, sim.stats()

    print(f"\n[surrogate tiled] precision {precision}: 32^3 and 32 x 32 x {32 * reps}", flush=True)
    small, st1 = run(1)
    big, stn = run(reps)
    assert st1["sur_fallbacks"] > 50
    assert stn["sur_fallbacks"] == reps * st1["sur_fallbacks"]
    assert stn["sur_voxels"] == reps * st1["sur_voxels"]
    for k in ("P", "Vc", "phi"):
        assert np.array_equal(big[k], np.tile(small[k], (1, 1, reps))), k


@pytest.fixture(scope="module")
def case_sur():
    """An oracle state after three oracle steps of the 32^3 workload (seed 9)
    with this step's fields solved, and a network: the oracle's initial
    parameters (seed 3) with biases ~ 0.3 N(0, 1), input statistics of the
    state's occupied voxels, output scales of a plausible update size."""
    from oracle import model as om
    print("\n[case_sur] oracle state, 32^3 seed 9", flush=True)
    tis = synth.make_tissue(32, 8, seed=9)
    sched = synth.bolus_schedule([0])
    osched = om.Schedule(times=sched.times, amts=sched.amts)
    s = om.init_state(tis.cell, tis.w, tis.seed, OP)
    for _ in range(3):
        s, _ = om.step(s, tis.w, osched, tis.seed, OP)
    K, G1, G2 = om.solve_fields(s, tis.w, osched, OP)
    s = om.State(s.L, K, G1, G2, s.P, s.Vc, s.phi, s.step)
    rng = np.random.default_rng(17)
    p = omlp.unpack(omlp.init_params(3))
    for k in p:
        if k.startswith("b"):
            p[k] = 0.3 * rng.standard_normal(p[k].shape)
    theta = omlp.pack(p).astype(np.float32).astype(np.float64)
    occ = s.L.ravel() != 0
    raw = np.stack([getattr(s, k).ravel() for k in ("K", "G1", "G2", "P", "Vc", "phi")], 1)[occ]
    sd = raw.std(0)
    stats = dict(in_mean=raw.mean(0).astype(np.float32),
                 in_scale=np.where(sd > 0, 1.0 / np.where(sd > 0, sd, 1.0), 1.0).astype(np.float32),
                 out_mean=np.array([1e-5, -2e-5, 5e-3], np.float32),
                 out_scale=np.array([3e-5, 4e-5, 2e-3], np.float32),
                 in_lo=raw.min(0).astype(np.float32), in_hi=raw.max(0).astype(np.float32))
    return tis, sched, s, theta, stats


@pytest.mark.parametrize("precision", [64, 32])
def test_surrogate_solve_end_in_the_ode_phase_is_the_separate_one(trained, precision):
    """In a full step the surrogate's kernel makes the solves' last
    x += alpha p on each run of voxels before it reads them (the plain
    kernel's case is in test_gpu_solve_end.py); run as separate phases, the
    solve makes it.  Two uneven replicates, three steps, a wide fallback
    margin (the fallback integrator reads the finished fields too): the
    same state and counts bit for bit."""
    tr, _ = trained
    net = tr.export()
    reps = []
    for shape, seed in (((12, 14, 10), 51), ((1, 20, 18), 52)):
        t = synth.make_tissue(shape, 4, seed=seed)
        sched = synth.bolus_schedule([0])
        reps.append((t.cell, t.w, t.seed, (sched.times, sched.amts)))
    params = hca.default_params(precision=precision)
    print(f"\n[surrogate solve end] precision {precision}", flush=True)
    with hca.Simulation(reps, params) as a, hca.Simulation(reps, params) as b:
        for sim in (a, b):
            sim.set_surrogate(net, 0.02)
        for n in range(3):
            a.step()
            b.run_phases(hca.PH_O2 | hca.PH_DRUGS)
            b.run_phases(hca.PH_ODE | hca.PH_CA | hca.PH_STATS | hca.PH_ADVANCE)
            for r in range(len(reps)):
                for k in ("L", "K", "G1", "G2", "P", "Vc", "phi"):
                    np.testing.assert_array_equal(a.field(k, r), b.field(k, r),
                                                  err_msg=f"step {n} replicate {r} {k}")
                np.testing.assert_equal(a.stats(r), b.stats(r), err_msg=f"step {n} replicate {r}")
        assert a.stats(0)["sur_voxels"] > 0
