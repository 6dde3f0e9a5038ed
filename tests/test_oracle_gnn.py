"""Pins of the surrogate network's CPU oracle (oracle/gnn.py) against things
other than itself: central finite differences for the hand-written backward
pass, a closed form of the message passing (mean degree 6 - 2 / L of the full
Chimera graph, from its coupler count 24 L^2 - 8 L), permutation and
readout invariants, and torch.optim.Adam for the optimiser step."""
import numpy as np
import pytest

import oracle
import oracle.gnn as G
import workloads


def _graphs(L, n, seed, missing=0.0):
    out = []
    for g in range(n):
        J = workloads.couplings(L, "pm7", seed, g)
        live = workloads.missing_mask(L, missing, seed, g) if missing else None
        out.append((L, live, J))
    return out


def _theta(seed, scale=0.15):
    return np.random.default_rng(seed).normal(0.0, scale, G.n_params())


def test_parameter_layout():
    assert G.n_params() == 4 * 64 + 2 * 64 + 5 * 64 + 4 * 64 - 4 * 64 + 3 * (64 * 193 + 64 * 129) + 65
    P = G.unpack(np.arange(G.n_params(), dtype=np.float64))
    assert P["W_m0"].shape == (64, 192) and P["W_h2"].shape == (64, 128) and P["b_out"].shape == (1,)


def test_graph_features():
    xn, xe, ei, ej, live = G.graph(2, None, np.ones(24 * 4 - 16, np.int8))
    assert xn.shape == (32, 5) and xe.shape == (80, 4)
    # every coupler is exactly one of intra-cell, along u = 0, along u = 1
    assert np.all(xe[:, 1:].sum(axis=1) == 1)
    assert int(xe[:, 1].sum()) == 16 * 4  # 16 intra couplers per cell
    assert np.all(ei < ej)


def test_backward_matches_central_differences():
    B = G.batch(_graphs(2, 3, 11, missing=0.1))
    labels = np.array([1.0, np.inf, -0.5])  # the infinite label is ignored
    theta = _theta(3)
    loss, grad, _ = G.loss_and_grad(theta, B, labels)
    rng = np.random.default_rng(5)
    # a few coordinates of every parameter block
    idx, o = [], 0
    for name, shp in G.param_shapes():
        n = int(np.prod(shp))
        idx += list(o + rng.choice(n, size=min(n, 6), replace=False))
        o += n
    h = 1e-6
    fd = []
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd.append((G.loss_and_grad(tp, B, labels)[0] - G.loss_and_grad(tm, B, labels)[0]) / (2 * h))
    fd = np.array(fd)
    an = grad[idx]
    rel = np.linalg.norm(fd - an) / np.linalg.norm(an)
    assert rel < 1e-6, rel


def test_mean_degree_closed_form():
    """h0 = 1, every message 1, h1 = in-degree, identity afterwards: y_hat is
    the mean degree 2 E / N = 6 - 2 / L of the full C_L."""
    for L in (2, 4, 5):
        B = G.batch(_graphs(L, 2, 1))
        P = G.unpack(np.zeros(G.n_params()))
        P["b_en"][:] = 1.0
        P["b_m0"][:] = 1.0
        P["W_h0"][:, 64:] = np.eye(64)
        for l in (1, 2):
            P["W_h" + str(l)][:, :64] = np.eye(64)
        P["w_out"][0] = 1.0
        theta = np.concatenate([P[name].ravel() for name, _ in G.param_shapes()])
        y, _ = G.forward(theta, B)
        assert np.allclose(y, 6.0 - 2.0 / L, rtol=0, atol=1e-12)


def test_batch_order_and_readout_invariants():
    gr = _graphs(3, 4, 21, missing=0.05)
    theta = _theta(8)
    y, _ = G.forward(theta, G.batch(gr))
    perm = [2, 0, 3, 1]
    yp, _ = G.forward(theta, G.batch([gr[i] for i in perm]))
    assert np.allclose(yp, y[perm], rtol=0, atol=1e-12)
    # the readout is affine in (w_out, b_out)
    P = G.unpack(theta.copy())
    P["b_out"][0] += 0.75
    t2 = np.concatenate([P[name].ravel() for name, _ in G.param_shapes()])
    y2, _ = G.forward(t2, G.batch(gr))
    assert np.allclose(y2, y + 0.75, atol=1e-12)


def test_bf16_rounding_and_mode():
    x = np.array([1.0, 1.00390625, 1.005859375, -3.14159, 65504.0])
    r = G.bf16(x)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0078125  # ties to even, then up
    assert abs(r[3] + 3.140625) < 1e-12
    B = G.batch(_graphs(2, 2, 4))
    theta = _theta(9)
    y64, _ = G.forward(theta, B)
    y16, _ = G.forward(theta, B, bf=True)
    assert np.linalg.norm(y16 - y64) / np.linalg.norm(y64) < 2e-2


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    th = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    p = torch.tensor(th.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 5):
        g = rng.normal(size=50)
        th, m, v = G.adam(th, m, v, g, step, 3e-3)
        opt.zero_grad()
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    assert np.allclose(th, p.detach().numpy(), rtol=0, atol=1e-12)


def _ranked_batch():
    # graphs 0 and 3 are parents; 1, 2 are children of 0 and 4 of 3; graph 5
    # has no parent and graph 2's label is missing
    gr = _graphs(2, 6, 13, missing=0.05)
    labels = np.array([0.4, 1.1, np.inf, -0.3, 0.9, 2.0])
    ref = [-1, 0, 0, -1, 3, -1]
    return G.batch(gr), labels, ref


def test_ranked_loss_backward_matches_central_differences():
    """The ranked loss (child against parent, plus w_abs times the plain
    loss): the hand-written gradient equals central differences of the
    loss."""
    B, labels, ref = _ranked_batch()
    theta = _theta(7)
    for w_abs in (0.0, 0.3):
        loss, grad, _ = G.loss_and_grad(theta, B, labels, ref=ref, w_abs=w_abs)
        rng = np.random.default_rng(9)
        idx, o = [], 0
        for name, shp in G.param_shapes():
            n = int(np.prod(shp))
            idx += list(o + rng.choice(n, size=min(n, 5), replace=False))
            o += n
        def fd(i, h):
            tp, tm = theta.copy(), theta.copy()
            tp[i] += h
            tm[i] -= h
            return (G.loss_and_grad(tp, B, labels, ref=ref, w_abs=w_abs)[0]
                    - G.loss_and_grad(tm, B, labels, ref=ref, w_abs=w_abs)[0]) / (2 * h)
        # a coordinate whose step crosses a ReLU kink gives differences that
        # change with the step: those (at most a few) are left out
        d1 = np.array([fd(i, 1e-6) for i in idx])
        d2 = np.array([fd(i, 2.5e-7) for i in idx])
        an = grad[idx]
        smooth = np.abs(d1 - d2) <= 1e-5 * np.maximum(np.abs(d2), 1e-3 * np.abs(an).max())
        assert smooth.sum() >= len(idx) - 4
        assert np.linalg.norm(d2[smooth] - an[smooth]) / np.linalg.norm(an[smooth]) < 1e-6


def test_ranked_loss_invariants():
    """Without the plain term the ranked loss sees only differences: a
    common shift of every label changes nothing, a common shift of every
    prediction changes nothing (so the output bias gets no gradient), and
    with no pairs the loss is w_abs times the plain loss."""
    B, labels, ref = _ranked_batch()
    theta = _theta(8)
    l0, g0, y0 = G.loss_and_grad(theta, B, labels, ref=ref, w_abs=0.0)
    l1, g1, _ = G.loss_and_grad(theta, B, labels + 3.25, ref=ref, w_abs=0.0)
    assert l1 == pytest.approx(l0, rel=1e-12) and np.allclose(g1, g0, rtol=1e-10, atol=1e-14)
    assert abs(G.unpack(g0)["b_out"][0]) < 1e-12 * max(1.0, np.abs(g0).max())
    t2 = theta.copy()
    t2[-1] += 5.0  # b_out shifts every prediction by 5
    l2, _, y2 = G.loss_and_grad(t2, B, labels, ref=ref, w_abs=0.0)
    assert np.allclose(y2, y0 + 5.0) and l2 == pytest.approx(l0, rel=1e-12)
    lp, gp, _ = G.loss_and_grad(theta, B, labels)
    ln, gn, _ = G.loss_and_grad(theta, B, labels, ref=[-1] * 6, w_abs=0.4)
    assert ln == pytest.approx(0.4 * lp, rel=1e-12) and np.allclose(gn, 0.4 * gp, rtol=1e-12, atol=1e-15)
    # a graph paired with an identical copy of itself: the predictions cancel,
    # the loss is the squared label difference and the gradient vanishes
    gr = _graphs(2, 1, 21)
    Bs = G.batch(gr + gr)
    ls, gs, _ = G.loss_and_grad(theta, Bs, np.array([0.5, 1.25]), ref=[-1, 0], w_abs=0.0)
    assert ls == pytest.approx(0.75 ** 2, rel=1e-12) and np.abs(gs).max() < 1e-12
