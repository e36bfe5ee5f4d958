"""Oracle: element-local MLP smoothing stage (test infrastructure only; see oracle/__init__).

The stage is not in the paper; it is defined by its formulas, written here plainly in FP64
(optionally emulating BF16 rounding of GEMM operands, RNE through float32):

Element features (one element e, n = (P+1)^d local nodes, local order i*(P+1)+j in 2D and
(i*(P+1)+m)*(P+1)+j in 3D, the vertical index fastest):
    r_e = R_e r          (R_e: element restriction of an assembled vector, the R_i of Sec. 5.3)
    s_e = ||r_e||_2
    X_e = [r_e / s_e, G_f / g_e for every factor field f, m_e / mean(m_e)],
          g_e = mean over the element's nodes of the trace (G_rr + G_ss, 3D also + G_tt);
          2D fields G_rr, G_rs, G_ss (5n inputs), 3D G_rr, G_tt, G_rs, G_ts, G_ss (7n inputs)
Network: 5n (2D) or 7n (3D) -> 128 -> 128 -> n with exact GELU(x) = x (1 + erf(x / sqrt 2)) / 2 on the two
hidden layers.  Output scaling: c_e = (s_e / a_e) y_e, a_e = mean of diag(A_e) (element matrix).
Assembly: c = W sum_e R_e^T c_e with W = (sum_e R_e R_e^T)^{-1} (the weight operator of Sec. 5.3:
the average over the elements sharing a node); zero on Dirichlet nodes.
Step: q = A c, alpha = (c.r)/(c.q), the energy-optimal step; accepted when alpha > 0 is finite
(then x += alpha c and the A-norm of the error drops by (c.r)^2 / (c.q)), otherwise skipped.  Training target: the element-local error determined by
the residual, t_e = (a_e / s_e) (R_e A R_e^T)^{-1} R_e r (the local solve of the Schwarz smoother,
Sec. 5.3); the raw global error R_e e is also available (``targets``).
Loss: mean over samples and outputs of (y - t)^2.  Adam (beta1 .9, beta2 .999, eps 1e-8).
"""
import math

import numpy as np
from scipy.special import erf

from .assemble import element_matrices
from .precision import bf16, f32  # noqa: F401  (BF16 emulation of the GEMM operands)

NH = 128


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def init_params(n_in, n_out, seed):
    """U(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases (NumPy generator; the library
    draws its own)."""
    rng = np.random.default_rng(seed)
    p = {}
    for k, (a, b) in enumerate([(n_in, NH), (NH, NH), (NH, n_out)], start=1):
        lim = 1.0 / math.sqrt(a)
        p[f"W{k}"] = rng.uniform(-lim, lim, (a, b))
        p[f"b{k}"] = np.zeros(b)
    return p


def forward(p, X, emulate=False):
    """Y = (GELU(GELU(X W1 + b1) W2 + b2)) W3 + b3.  emulate: BF16 GEMM operands, FP32 rest."""
    q = bf16 if emulate else (lambda a: a)
    Z1 = q(X) @ q(p["W1"]) + p["b1"]
    H1 = gelu(Z1)
    Z2 = q(H1) @ q(p["W2"]) + p["b2"]
    H2 = gelu(Z2)
    Y = q(H2) @ q(p["W3"]) + p["b3"]
    if emulate:
        Z1, H1, Z2, H2, Y = f32(Z1), f32(H1), f32(Z2), f32(H2), f32(Y)
    return Y, dict(X=X, Z1=Z1, H1=H1, Z2=Z2, H2=H2)


def mse(Y, T):
    d = Y - T
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(p, cache, dY, emulate=False):
    """Gradients of the loss for every parameter (no input gradient)."""
    q = bf16 if emulate else (lambda a: a)
    X, Z1, H1, Z2, H2 = (cache[k] for k in ("X", "Z1", "H1", "Z2", "H2"))
    g = {}
    g["W3"] = q(H2).T @ q(dY)
    g["b3"] = dY.sum(axis=0)
    dH2 = q(dY) @ q(p["W3"]).T
    dZ2 = dH2 * gelu_grad(Z2)
    g["W2"] = q(H1).T @ q(dZ2)
    g["b2"] = dZ2.sum(axis=0)
    dH1 = q(dZ2) @ q(p["W2"]).T
    dZ1 = dH1 * gelu_grad(Z1)
    g["W1"] = q(X).T @ q(dZ1)
    g["b1"] = dZ1.sum(axis=0)
    return g


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new params and moments."""
    out, mo, vo = {}, {}, {}
    for k in p:
        mo[k] = b1 * m[k] + (1 - b1) * g[k]
        vo[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = mo[k] / (1 - b1 ** t)
        vh = vo[k] / (1 - b2 ** t)
        out[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return out, mo, vo


def cosine_lr(lr0, step, total_steps):
    """Learning rate of Adam step ``step`` (counted from 1) out of ``total_steps``: cosine decay
    from lr0, lr0 (1 + cos(pi (step - 1) / total_steps)) / 2."""
    return lr0 * 0.5 * (1.0 + math.cos(math.pi * (step - 1) / total_steps))


def train_full_batch(p, X, T, steps, lr0, total_steps=None, emulate=True):
    """``steps`` Adam steps on the whole set (rows in order, no shuffling) with the cosine
    schedule over ``total_steps`` (default: steps).  Returns the parameters and the loss before
    each step."""
    total_steps = steps if total_steps is None else total_steps
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    losses = []
    for t in range(1, steps + 1):
        Y, cache = forward(p, X, emulate)
        loss, dY = mse(Y, T)
        losses.append(loss)
        g = backward(p, cache, dY, emulate)
        p, m, v = adam(p, g, m, v, t, cosine_lr(lr0, t, total_steps))
    return p, losses


# ---- element features and the smoothing stage ------------------------------------------------
def element_scales(mesh):
    """g_e (feature scale: element mean of the trace of the factor tensor, G_rr + G_ss in 2D,
    G_rr + G_tt + G_ss in 3D), mean mass, and a_e = mean of diag(A_e) for every element."""
    E = mesh.E
    tr = mesh.Grr.reshape(E, -1) + mesh.Gss.reshape(E, -1)
    if mesh.dim == 3:
        tr = tr + mesh.Gtt.reshape(E, -1)
    g = tr.mean(axis=1)
    mm = mesh.mass.reshape(E, -1).mean(axis=1)
    Ae = element_matrices(mesh)
    a = np.einsum("ekk->ek", Ae).mean(axis=1)
    return g, mm, a


def features(mesh, r, scales=None):
    """X and s_e for an assembled residual r: per element [r_e / s_e, every factor field / g_e,
    m_e / mean(m_e)], the fields in the order of mesh.fields() (2D: G_rr, G_rs, G_ss, so
    5n columns; 3D: G_rr, G_tt, G_rs, G_ts, G_ss, so 7n columns; G_rt vanishes because x and y
    are affine)."""
    E = mesh.E
    g, mm, _ = scales if scales is not None else element_scales(mesh)
    re = np.asarray(r, dtype=np.float64)[mesh.l2g]
    s = np.sqrt((re * re).sum(axis=1))
    safe = np.where(s > 0, s, 1.0)
    rn = np.where(s[:, None] > 0, re / safe[:, None], 0.0)
    geo = [F.reshape(E, -1) / g[:, None] for F in mesh.fields()]
    X = np.concatenate([rn] + geo + [mesh.mass.reshape(E, -1) / mm[:, None]], axis=1)
    return X, s


def targets(mesh, e, s, scales=None):
    _, _, a = scales if scales is not None else element_scales(mesh)
    ee = np.asarray(e, dtype=np.float64)[mesh.l2g]
    safe = np.where(s > 0, s, 1.0)
    return np.where(s[:, None] > 0, (a / safe)[:, None] * ee, 0.0)


def local_targets(mesh, A, r, s, scales=None):
    """Targets from the element-block solves: t_e = (a_e / s_e) (R_e A R_e^T)^{-1} R_e r, the
    local solve of the Schwarz smoother of Sec. 5.3 (A: the masked assembled matrix)."""
    _, _, a = scales if scales is not None else element_scales(mesh)
    Ad = A.tocsr()
    r = np.asarray(r, dtype=np.float64)
    out = np.zeros((mesh.E, mesh.l2g.shape[1]))
    for e in range(mesh.E):
        idx = mesh.l2g[e]
        if s[e] > 0:
            Ae = Ad[idx][:, idx].toarray()
            out[e] = (a[e] / s[e]) * np.linalg.solve(Ae, r[idx])
    return out


def multiplicity(mesh):
    return np.bincount(mesh.l2g.ravel(), minlength=mesh.N).astype(np.float64)


def correction(mesh, p, r, emulate=True, scales=None):
    """Assembled, weighted correction c for residual r (zero on Dirichlet nodes)."""
    sc = scales if scales is not None else element_scales(mesh)
    X, s = features(mesh, r, sc)
    Y, _ = forward(p, X, emulate)
    a = sc[2]
    ce = (s / a)[:, None] * Y
    c = np.bincount(mesh.l2g.ravel(), weights=ce.ravel(), minlength=mesh.N) / multiplicity(mesh)
    c[mesh.dirichlet_nodes()] = 0.0
    return c


def stage(A, mesh, p, b, x, emulate=True, scales=None):
    """One learned smoothing stage on the assembled system A x = b; returns (x, accepted)."""
    r = b - A @ x
    c = correction(mesh, p, r, emulate, scales)
    q = A @ c
    cq = c @ q
    alpha = (c @ r) / cq if cq != 0 else float("nan")
    ok = bool(np.isfinite(alpha) and alpha > 0)
    return (x + alpha * c if ok else x), ok
