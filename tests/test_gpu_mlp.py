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
from paper_2105_00448_amd import hca, synth

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
