"""Reference message-passing preconditioner network.  TEST INFRASTRUCTURE ONLY.

numpy, float64, written from the network's definition (below); the GPU library's
forward/backward kernels are checked against it, and it is checked against central
finite differences.  With ``bf16=True`` the weights and every dense-layer input are
rounded to bfloat16 (round-to-nearest-even on the float32 bit pattern), as the GPU
does; the backward pass treats that rounding as the identity (straight-through).

Definition (a learned "diagonal plus neighbour" approximate inverse of a Stieltjes
matrix A -- SPD with non-positive off-diagonal entries, like every diffusion matrix --
with a symmetric pattern; hi = leading binary64 component of the DD values):
  minv_i = 1 / hi(a_ii);  w_ij = -hi(a_ij) / sqrt(hi(a_ii) hi(a_jj))  (i != j), float32
  features f_i = [sum_j w_ij, sum_j w_ij^2, deg_i / 8, 1]            (float32)
  h0 = relu(f W0 + b0)                                                 (4 -> 64)
  layer l = 1..3:  m_i = sum_j w_ij h_j  (row order);  h = relu(h Ws_l + m Wn_l + b_l)
  u_i = h_i . wu + bu;   v_ij = sum_k qv_k (h_ik h_jk) + bv               (v_ij = v_ji)
  g_ij = tanh(v_ij)^2 in [0, 1);  c_ij = g_ij w_ij;  delta_i = log(1 + u_i^2) >= 0
  M_ii = (1 + delta_i) minv_i;  M_ij = c_ij sqrt(minv_i minv_j)
that is M = S (I + Delta + G o W) S with S = D^-1/2: a damped first-order Neumann
approximation of A^-1 = S (I - W)^-1 S (g = 1, delta = 0 is exactly I + W).  M is SPD:
W >= 0 entrywise with spectral radius rho(W) < 1 (I - W = S A S is SPD), so
0 <= G o W <= W entrywise has rho(G o W) <= rho(W) < 1, every eigenvalue of G o W
exceeds -1, and I + Delta + G o W with Delta >= 0 is positive definite.  With every
weight zero (and zero biases) M is exactly the Jacobi inverse diagonal.
Training loss of a pair (r, e):  L = (M r - e)^T A (M r - e) / e^T A e.

Parameter vector (float32, this order): W0 (4x64 row-major), b0 (64), then for l = 1..3:
Ws_l (64x64), Wn_l (64x64), b_l (64); then wu (64), bu (1), qv (64), bv (1).
"""
import numpy as np

HIDDEN = 64
NFEAT = 4


def param_shapes(hidden=HIDDEN):
    shapes = [("W0", (NFEAT, hidden)), ("b0", (hidden,))]
    for l in range(1, 4):
        shapes += [("Ws%d" % l, (hidden, hidden)), ("Wn%d" % l, (hidden, hidden)), ("b%d" % l, (hidden,))]
    shapes += [("wu", (hidden,)), ("bu", (1,)), ("qv", (hidden,)), ("bv", (1,))]
    return shapes


def n_params(hidden=HIDDEN):
    return sum(int(np.prod(s)) for _, s in param_shapes(hidden))


def unpack(theta, hidden=HIDDEN):
    out, o = {}, 0
    for name, shp in param_shapes(hidden):
        k = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return out


def pack(p, hidden=HIDDEN):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in param_shapes(hidden)])


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even) and return them as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


class Graph:
    """Pattern, edge weights and features of one matrix (hi components)."""

    def __init__(self, row_ptr, col_idx, a_hi):
        self.rp = np.asarray(row_ptr, dtype=np.int64)
        self.ci = np.asarray(col_idx, dtype=np.int64)
        self.n = self.rp.size - 1
        a = np.asarray(a_hi, dtype=np.float64)
        self.rows = np.repeat(np.arange(self.n), np.diff(self.rp))
        diag = np.zeros(self.n)
        dmask = self.rows == self.ci
        diag[self.rows[dmask]] = a[dmask]
        self.minv = 1.0 / diag
        self.offd = ~dmask
        w = np.zeros(self.ci.size)
        w[self.offd] = -a[self.offd] / np.sqrt(diag[self.rows[self.offd]] * diag[self.ci[self.offd]])
        self.w = w.astype(np.float32).astype(np.float64)
        deg = np.bincount(self.rows[self.offd], minlength=self.n)
        s1 = np.bincount(self.rows, weights=self.w, minlength=self.n)
        s2 = np.bincount(self.rows, weights=self.w * self.w, minlength=self.n)
        f = np.stack([s1, s2, deg / 8.0, np.ones(self.n)], axis=1)
        self.f = f.astype(np.float32).astype(np.float64)
        self.a_hi = a

    def aggregate(self, H):
        """m_i = sum_j w_ij H_j."""
        out = np.zeros((self.n, H.shape[1]))
        np.add.at(out, self.rows, self.w[:, None] * H[self.ci])
        return out

    def spmv(self, vals, x):
        out = np.zeros(self.n)
        np.add.at(out, self.rows, vals * x[self.ci])
        return out


def forward(g, theta, bf=False):
    """Returns (M values on the pattern, cache)."""
    p = unpack(theta)
    q = (lambda x: bf16(x)) if bf else (lambda x: x)
    c = {"p": p}
    H = np.maximum(q(g.f) @ q(p["W0"]) + p["b0"], 0.0)
    c["H"] = [H]
    c["Mg"] = [None]
    for l in range(1, 4):
        Mg = g.aggregate(H)
        H = np.maximum(q(H) @ q(p["Ws%d" % l]) + q(Mg) @ q(p["Wn%d" % l]) + p["b%d" % l], 0.0)
        c["H"].append(H)
        c["Mg"].append(Mg)
    Hq = q(H)
    u = Hq @ q(p["wu"]) + p["bu"][0]
    v = (Hq[g.rows] * Hq[g.ci]) @ q(p["qv"]) + p["bv"][0]
    th = np.tanh(v)
    cc = np.where(g.offd, th * th * g.w, 0.0)
    delta = np.log1p(u * u)
    diag = 1.0 + delta
    M = np.where(g.offd, cc * np.sqrt(g.minv[g.rows] * g.minv[g.ci]), 0.0)
    dmask = ~g.offd
    M[dmask] = diag[g.rows[dmask]] * g.minv[g.rows[dmask]]
    c.update(u=u, v=v, cc=cc, diag=diag, Hq=Hq, q=q)
    return M, c


def loss(g, M, r, e):
    """L = (M r - e)^T A (M r - e) / e^T A e, with A = the graph's hi values."""
    d = g.spmv(M, r) - e
    Ad = g.spmv(g.a_hi, d)
    Ae = g.spmv(g.a_hi, e)
    E = float(e @ Ae)
    return float(d @ Ad) / E, 2.0 * Ad / E


def backward(g, theta, r, e, bf=False):
    """Loss and gradient with respect to the parameter vector."""
    M, c = forward(g, theta, bf)
    L, gy = loss(g, M, r, e)
    p, q = c["p"], c["q"]
    rows, ci = g.rows, g.ci
    G = gy * r * g.minv                        # dL/d diag_i
    dc = np.where(g.offd, gy[rows] * r[ci] * np.sqrt(g.minv[rows] * g.minv[ci]), 0.0)
    th = np.tanh(c["v"])
    dv = np.where(g.offd, dc * g.w * 2.0 * th * (1.0 - th * th), 0.0)
    du = G * 2.0 * c["u"] / (1.0 + c["u"] * c["u"])
    grads = {k: np.zeros_like(v) for k, v in p.items()}
    Hq = c["Hq"]
    qv = q(p["qv"])
    grads["wu"] = Hq.T @ du
    grads["bu"] = np.array([du.sum()])
    grads["qv"] = (dv[:, None] * Hq[rows] * Hq[ci]).sum(axis=0)
    grads["bv"] = np.array([dv.sum()])
    dH = du[:, None] * q(p["wu"])[None, :]
    np.add.at(dH, rows, dv[:, None] * qv[None, :] * Hq[ci])
    np.add.at(dH, ci, dv[:, None] * qv[None, :] * Hq[rows])
    for l in range(3, 0, -1):
        H, Hprev, Mg = c["H"][l], c["H"][l - 1], c["Mg"][l]
        dZ = dH * (H > 0)
        grads["Ws%d" % l] = q(Hprev).T @ dZ
        grads["Wn%d" % l] = q(Mg).T @ dZ
        grads["b%d" % l] = dZ.sum(axis=0)
        dHprev = dZ @ q(p["Ws%d" % l]).T
        dMg = dZ @ q(p["Wn%d" % l]).T
        dH = dHprev + g.aggregate(dMg)   # symmetric weights and pattern: transpose = itself
    dZ = dH * (c["H"][0] > 0)
    grads["W0"] = q(g.f).T @ dZ
    grads["b0"] = dZ.sum(axis=0)
    return L, pack(grads)


def init_params(seed, scale=0.1):
    """Small random weights, zero biases (float32 values)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in param_shapes():
        if name.startswith("b"):
            p[name] = np.zeros(shp)
        else:
            fan_in = shp[0] if len(shp) == 2 else HIDDEN
            p[name] = rng.normal(0.0, scale / np.sqrt(fan_in), size=shp)
    return pack(p).astype(np.float32).astype(np.float64)


def adam(theta, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, bias-corrected), float64.  Returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
