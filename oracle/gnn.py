"""CPU ORACLE for the hardness surrogate -- TEST INFRASTRUCTURE ONLY.

Plain float64 numpy reference of the edge message-passing network that
ranks proposed coupler mutations inside the instance search (the search
itself is Algorithm 1, Sec. II.A; the network has no counterpart in the
paper: its definition below is the reading used throughout).  Only tests/
and the smoke check may import it.

Graph of one instance (L, live, J) on Chimera C_L (Appendix A, Fig. 8):
  node v (site id 8 (L r + c) + 4 u + k): features (r / L, c / L, u, k / 3, live)
  undirected coupler q = (i, j), i < j, canonical order: features
      (J_q / 7, intra-cell, inter-cell along u = 0, inter-cell along u = 1)
  directed edges 2 q (i -> j) and 2 q + 1 (j -> i); in(v) = edges with dst v.
Network (width D = 64, three layers, ReLU):
  h0_v = W_en x_v + b_en                 m0_e = W_ee f_q(e) + b_ee
  layer l:  m_e <- relu(W_m [h_src(e); h_dst(e); m_e] + b_m)
            h_v <- relu(W_h [h_v; sum_{e in in(v)} m_e] + b_h)
  y_hat = w . mean_{live v} h_v + b_out
Loss: mean over graphs with a finite label of (y_hat - y)^2 (y = ln TTS).
Ranked loss (a child instance against its parent, one coupler apart): with
ref[g] the index of graph g's parent in the batch (-1: none),
  mean over pairs (g, p = ref[g]) with p in range, p != g and both labels
  finite of ((y_hat_g - y_hat_p) - (y_g - y_p))^2  +  w_abs * (the loss above)
so that the network learns the change of ln TTS one mutation makes.
Optimiser: Adam (Kingma and Ba, ICLR 2015) with bias correction.

With bf16=True every value the GPU kernels hold in bfloat16 is rounded to
bfloat16 (round to nearest even) at the same points: the node and edge
states H, M and the message sums S fed to the matrix products, the weight
matrices W_m, W_h, and the pre-activation gradients dZ fed to the backward
products; everything else stays float64.
"""
import numpy as np

from . import edges as _chimera_edges

D = 64
NODE_F = 5
EDGE_F = 4
LAYERS = 3


def param_shapes():
    shapes = [("W_en", (D, NODE_F)), ("b_en", (D,)), ("W_ee", (D, EDGE_F)), ("b_ee", (D,))]
    for l in range(LAYERS):
        shapes += [(f"W_m{l}", (D, 3 * D)), (f"b_m{l}", (D,)), (f"W_h{l}", (D, 2 * D)),
                   (f"b_h{l}", (D,))]
    shapes += [("w_out", (D,)), ("b_out", (1,))]
    return shapes


def n_params():
    return sum(int(np.prod(s)) for _, s in param_shapes())


def unpack(theta):
    out, o = {}, 0
    for name, shp in param_shapes():
        n = int(np.prod(shp))
        out[name] = theta[o:o + n].reshape(shp)
        o += n
    return out


def bf16(x):
    """Round to bfloat16 (nearest even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def graph(L, live, J):
    """Node features (N, 5), edge features (E, 4), endpoints i < j (E,)."""
    N = 8 * L * L
    ei, ej = _chimera_edges(L)
    live = np.ones(N, np.uint8) if live is None else np.asarray(live, np.uint8)
    v = np.arange(N)
    cell, u, k = v // 8, (v // 4) % 2, v % 4
    r, c = cell // L, cell % L
    xn = np.stack([r / L, c / L, u, k / 3.0, live.astype(np.float64)], axis=1)
    ci, cj = ei // 8, ej // 8
    intra = (ci == cj).astype(np.float64)
    inter_u0 = ((ci != cj) & (((ei // 4) % 2) == 0)).astype(np.float64)
    inter_u1 = ((ci != cj) & (((ei // 4) % 2) == 1)).astype(np.float64)
    Jq = np.asarray(J, np.float64)
    # couplers touching a missing site carry no interaction
    Jq = np.where((live[ei] == 1) & (live[ej] == 1), Jq, 0.0)
    xe = np.stack([Jq / 7.0, intra, inter_u0, inter_u1], axis=1)
    return xn, xe, ei.astype(np.int64), ej.astype(np.int64), live


def batch(graphs):
    """Concatenates per-instance graphs (list of (L, live, J), same L)."""
    parts = [graph(*g) for g in graphs]
    N = parts[0][0].shape[0]
    E = parts[0][1].shape[0]
    xn = np.concatenate([p[0] for p in parts])
    xe = np.concatenate([p[1] for p in parts])
    src = np.empty(2 * E * len(parts), np.int64)
    dst = np.empty_like(src)
    for g, p in enumerate(parts):
        i, j = p[2] + g * N, p[3] + g * N
        a = g * 2 * E
        src[a:a + 2 * E:2], dst[a:a + 2 * E:2] = i, j
        src[a + 1:a + 2 * E:2], dst[a + 1:a + 2 * E:2] = j, i
    live = np.concatenate([p[4] for p in parts]).astype(np.float64)
    return dict(xn=xn, xe=xe, src=src, dst=dst, live=live, G=len(parts), N=N, E=E)


def _r(x, on):
    return bf16(x) if on else x


def forward(theta, B, bf=False):
    """y_hat (G,) and the intermediates the backward pass needs."""
    P = unpack(np.asarray(theta, np.float64))
    G, N, E = B["G"], B["N"], B["E"]
    H = _r(B["xn"] @ P["W_en"].T + P["b_en"], bf)
    m0 = B["xe"] @ P["W_ee"].T + P["b_ee"]
    M = _r(np.repeat(m0, 2, axis=0), bf)
    src, dst = B["src"], B["dst"]
    cache = dict(layers=[], H0=H, M0=M)
    for l in range(LAYERS):
        Wm, Wh = _r(P[f"W_m{l}"], bf), _r(P[f"W_h{l}"], bf)
        Xe = np.concatenate([H[src], H[dst], M], axis=1)
        Zm = Xe @ Wm.T + P[f"b_m{l}"]
        Mn = _r(np.maximum(Zm, 0.0), bf)
        S = np.zeros((G * N, D))
        np.add.at(S, dst, Mn)
        S = _r(S, bf)
        Xn = np.concatenate([H, S], axis=1)
        Zh = Xn @ Wh.T + P[f"b_h{l}"]
        Hn = _r(np.maximum(Zh, 0.0), bf)
        cache["layers"].append(dict(Xe=Xe, Zm=Zm, Xn=Xn, Zh=Zh, Wm=Wm, Wh=Wh))
        H, M = Hn, Mn
    live = B["live"].reshape(G, N)
    nl = live.sum(axis=1)
    mean = (H.reshape(G, N, D) * live[:, :, None]).sum(axis=1) / nl[:, None]
    y = mean @ P["w_out"] + P["b_out"][0]
    cache.update(H=H, mean=mean, nl=nl)
    return y, cache


def loss_and_grad(theta, B, labels, bf=False, ref=None, w_abs=1.0):
    """(loss, gradient (flat, like theta), y_hat); labels that are not
    finite are left out of the mean.  With ref, the ranked loss (module
    docstring) with weight w_abs on the plain term."""
    theta = np.asarray(theta, np.float64)
    P = unpack(theta)
    y, c = forward(theta, B, bf)
    G, N = B["G"], B["N"]
    labels = np.asarray(labels, np.float64)
    ok = np.isfinite(labels)
    nv = max(1, int(ok.sum()))
    diff = np.where(ok, y - np.where(ok, labels, 0.0), 0.0)
    loss = float((diff ** 2).sum() / nv)
    dy = 2.0 * diff / nv
    if ref is not None:
        ref = [int(r) for r in ref]
        pairs = [(g, ref[g]) for g in range(G) if 0 <= ref[g] < G and ref[g] != g and ok[g] and ok[ref[g]]]
        npair = max(1, len(pairs))
        loss *= w_abs
        dy = dy * w_abs
        for g, p_ in pairs:
            d = (y[g] - y[p_]) - (labels[g] - labels[p_])
            loss += d * d / npair
            dy[g] += 2.0 * d / npair
            dy[p_] -= 2.0 * d / npair
        loss = float(loss)
    g = {k: np.zeros_like(v) for k, v in P.items()}
    g["w_out"] = dy @ c["mean"]
    g["b_out"][0] = dy.sum()
    live = B["live"].reshape(G, N)
    dH = ((dy / c["nl"])[:, None, None] * P["w_out"][None, None, :] * live[:, :, None]).reshape(G * N, D)
    src, dst = B["src"], B["dst"]
    dM = np.zeros((G * 2 * B["E"], D))
    for l in reversed(range(LAYERS)):
        L_ = c["layers"][l]
        dZh = dH * (L_["Zh"] > 0)
        g[f"b_h{l}"] = dZh.sum(axis=0)
        dZh_b = _r(dZh, bf)
        g[f"W_h{l}"] = dZh_b.T @ L_["Xn"]
        dXn = dZh_b @ L_["Wh"]
        dH_prev = dXn[:, :D].copy()
        dS = dXn[:, D:]
        dMn = dM + dS[dst]
        dZm = dMn * (L_["Zm"] > 0)
        g[f"b_m{l}"] = dZm.sum(axis=0)
        dZm_b = _r(dZm, bf)
        g[f"W_m{l}"] = dZm_b.T @ L_["Xe"]
        dXe = dZm_b @ L_["Wm"]
        np.add.at(dH_prev, src, dXe[:, :D])
        np.add.at(dH_prev, dst, dXe[:, D:2 * D])
        dM = dXe[:, 2 * D:]
        dH = dH_prev
    g["W_en"] = dH.T @ B["xn"]
    g["b_en"] = dH.sum(axis=0)
    dm0 = dM[0::2] + dM[1::2]
    g["W_ee"] = dm0.T @ B["xe"]
    g["b_ee"] = dm0.sum(axis=0)
    flat = np.concatenate([g[name].ravel() for name, _ in param_shapes()])
    return loss, flat, y


def adam(theta, m, v, grad, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
