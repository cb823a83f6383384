"""Learned post-smoothing correction: network, training step and the guarded
outer iteration (test infrastructure, like the rest of this package).

The paper has no learned component; this module states the added method so
that the GPU path can be checked against it.

Correction.  After the V-cycle (post-smoothing on the finest level) the
residual r = b - A x_post is formed; per element E the network maps the
3^d patch of elements around E to a correction of x_E:

* input channels of one element F: its n_b residual coefficients divided by
  the global RMS of the velocity (s_u) or pressure (s_p) coefficients of r,
  then log10 of the element mean of mu (the (0, 0) entry of M_mu, the basis
  being orthonormal); n_b + 1 channels;
* patch: offsets o in {-1, 0, 1}^d, axis 0 fastest; elements outside a
  non-periodic wall contribute zero channels, periodic axes wrap;
* layers: a1 = W1 z_patch + b1 (H outputs), h1 = relu(a1),
  a2 = W2 h1 + b2, h2 = relu(a2), y = W3 h2 + b3 (n_b outputs);
* output: dx_E = y * s_f * c_f per coefficient, f the coefficient's field
  (velocity or pressure), c_f a per-field constant measured on the training
  data (RMS of e / s_f).

Training.  Pairs (r, e) come from plain V-cycles on A x* = b for random smooth
x*, e = x* - x_post with the kernel removed.  Loss: the mean squared
difference between y and e / (s_f c_f).  Adam (Kingma and Ba, 2015) on FP32
master weights.

BF16 emulation.  ``bf16`` rounds float32 to the nearest bfloat16 (ties to
even).  The reduced-precision network rounds the input channels, weights and
hidden activations to bfloat16, accumulates products in float32, and adds the
biases in float32.

Minimal-residual step.  With z = V(v) the cycle's result for the vector v
it is applied to, r' = v - A z (in the cycle's precision) and dx the
network's correction of r', the preconditioned result is z + w dx with
w = <r', A dx> / ||A dx||^2 (0 when A dx = 0), inner products in the
variables of the diagonally scaled system, A dx in the cycle's precision.
The step minimises ||r' - w A dx|| over w, so the correction never raises the
residual the cycle leaves.  It serves both outer iterations below; FGMRES
(flexible, right-preconditioned) takes z + w dx as its direction.

Guard (iterative refinement).  The first two outer iterations are plain and give
rho_plain = (||r_2|| / ||r_0||)^(1/2).  Later iterations apply the
correction; with c_k = ||r_k|| / ||r_{k-1}||, the correction is switched off
for the rest of the solve when c_k > 1 once or c_k > 1.1 rho_plain in two
consecutive iterations, and the iteration that triggered it is replaced by
its plain result.
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# bfloat16 rounding
# ---------------------------------------------------------------------------
def bf16(x):
    """Round to the nearest bfloat16 value (ties to even), returned as float32."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    nan = np.isnan(a)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    out = r.astype(np.uint32).view(np.float32).reshape(a.shape)
    if nan.any():
        out = out.copy()
        out[nan] = np.nan
    return out


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def n_offsets(d):
    return 3 ** d


def offsets(d):
    """Patch offsets, axis 0 fastest."""
    out = []
    for i in range(3 ** d):
        o, t = [], i
        for _ in range(d):
            o.append(t % 3 - 1)
            t //= 3
        out.append(tuple(o))
    return out


def init_params(d, nb, H, seed):
    """He-normal weights, zero biases (FP64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    K = n_offsets(d) * (nb + 1)
    return {
        "W1": rng.standard_normal((H, K)) * np.sqrt(2.0 / K),
        "b1": np.zeros(H),
        "W2": rng.standard_normal((H, H)) * np.sqrt(2.0 / H),
        "b2": np.zeros(H),
        "W3": rng.standard_normal((nb, H)) * np.sqrt(1.0 / H),
        "b3": np.zeros(nb),
    }


def element_channels(r, logmu, d, nq, s=None):
    """(NE, nb+1) input channels and the scales (s_u, s_p)."""
    nb = (d + 1) * nq
    R = np.asarray(r, dtype=np.float64).reshape(-1, nb)
    if s is None:
        su = np.sqrt(np.mean(R[:, :d * nq] ** 2))
        sp = np.sqrt(np.mean(R[:, d * nq:] ** 2))
        s = (su if su > 0 else 1.0, sp if sp > 0 else 1.0)
    Z = np.empty((R.shape[0], nb + 1))
    Z[:, :d * nq] = R[:, :d * nq] / s[0]
    Z[:, d * nq:nb] = R[:, d * nq:] / s[1]
    Z[:, nb] = logmu
    return Z, s


def patches(Z, shape, periodic):
    """(NE, 3^d * C) patch matrix of an element field Z (NE, C) on a grid of
    the given shape (axis 0 fastest), zero outside non-periodic walls."""
    d = len(shape)
    C = Z.shape[1]
    grid = Z.reshape(tuple(reversed(shape)) + (C,))        # numpy axes: (axis d-1, ..., axis 0, C)
    out = []
    for o in offsets(d):
        g = grid
        for k in range(d):
            ax = d - 1 - k
            if periodic[k]:
                g = np.roll(g, -o[k], axis=ax)
            elif o[k] != 0:
                shifted = np.zeros_like(g)
                sl_dst = [slice(None)] * (d + 1)
                sl_src = [slice(None)] * (d + 1)
                if o[k] > 0:
                    sl_dst[ax], sl_src[ax] = slice(0, shape[k] - 1), slice(1, shape[k])
                else:
                    sl_dst[ax], sl_src[ax] = slice(1, shape[k]), slice(0, shape[k] - 1)
                shifted[tuple(sl_dst)] = g[tuple(sl_src)]
                g = shifted
        out.append(g.reshape(-1, C))
    return np.concatenate(out, axis=1)


def forward(params, X, emulate_bf16=False):
    """Layer values for patch rows X (N, K); FP64, or the BF16 emulation."""
    if emulate_bf16:
        Xq = bf16(X)
        W1, W2, W3 = (bf16(params[k]) for k in ("W1", "W2", "W3"))
        b1, b2, b3 = (params[k].astype(np.float32) for k in ("b1", "b2", "b3"))
        a1 = Xq @ W1.T + b1
        h1 = bf16(np.maximum(a1, 0))
        a2 = h1 @ W2.T + b2
        h2 = bf16(np.maximum(a2, 0))
        y = h2 @ W3.T + b3
        return {"X": Xq, "a1": a1, "h1": h1, "a2": a2, "h2": h2, "y": y}
    a1 = X @ params["W1"].T + params["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ params["W2"].T + params["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ params["W3"].T + params["b3"]
    return {"X": X, "a1": a1, "h1": h1, "a2": a2, "h2": h2, "y": y}


def backward(params, cache, dy, emulate_bf16=False):
    """Gradients of sum(dy * y) with respect to every parameter."""
    if emulate_bf16:
        dy = bf16(dy)
        W2, W3 = bf16(params["W2"]), bf16(params["W3"])
        g = {"W3": dy.T @ cache["h2"], "b3": dy.sum(0)}
        dh2 = bf16(dy @ W3)
        da2 = np.where(cache["a2"] > 0, dh2, 0).astype(np.float32)
        g["W2"], g["b2"] = da2.T @ cache["h1"], da2.sum(0)
        dh1 = bf16(da2 @ W2)
        da1 = np.where(cache["a1"] > 0, dh1, 0).astype(np.float32)
        g["W1"], g["b1"] = da1.T @ cache["X"], da1.sum(0)
        return g
    g = {"W3": dy.T @ cache["h2"], "b3": dy.sum(0)}
    da2 = (dy @ params["W3"]) * (cache["a2"] > 0)
    g["W2"], g["b2"] = da2.T @ cache["h1"], da2.sum(0)
    da1 = (da2 @ params["W2"]) * (cache["a1"] > 0)
    g["W1"], g["b1"] = da1.T @ cache["X"], da1.sum(0)
    return g


def loss_and_grad(params, X, T, emulate_bf16=False):
    """Mean squared error between y and targets T (N, nb), and its gradient."""
    c = forward(params, X, emulate_bf16)
    diff = c["y"] - T
    loss = float(np.mean(np.asarray(diff, dtype=np.float64) ** 2))
    dy = 2.0 * diff / diff.size
    return loss, backward(params, c, dy, emulate_bf16)


class Adam:
    """Adam with bias correction (Kingma and Ba, 2015), state in FP64."""

    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = {k: np.zeros_like(v) for k, v in params.items()}
        self.v = {k: np.zeros_like(v) for k, v in params.items()}
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        for k in params:
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * grads[k]
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * grads[k] ** 2
            mh = self.m[k] / (1 - self.b1 ** self.t)
            vh = self.v[k] / (1 - self.b2 ** self.t)
            params[k] = params[k] - self.lr * mh / (np.sqrt(vh) + self.eps)
        return params


# ---------------------------------------------------------------------------
# the correction on a whole grid
# ---------------------------------------------------------------------------
class Grid:
    """Finest-level geometry needed by the network."""

    def __init__(self, d, n, p, periodic, logmu):
        self.d, self.n, self.p = d, n, p
        self.nq = (p + 1) ** d
        self.nb = (d + 1) * self.nq
        self.periodic = tuple(periodic)
        self.logmu = np.asarray(logmu, dtype=np.float64)


def grid_of(hier):
    """Network geometry of a hierarchy's finest level (log10 of the element
    mean of mu from the (0, 0) entry of each M_mu block)."""
    prob = hier.prob
    fine = hier.fine
    nq = fine.nq
    Mmu = fine.ops["Mmu"]
    mu_e = np.array([Mmu[E * nq, E * nq] for E in range(fine.NE)])
    per = [b == "periodic" for b in prob.bc]
    return Grid(prob.dim, fine.n, prob.p, per, np.log10(mu_e))


def correction(params, cvec, g, r, emulate_bf16=False):
    """dx for residual r (element-major) on grid g."""
    Z, s = element_channels(r, g.logmu, g.d, g.nq)
    X = patches(Z, (g.n,) * g.d, g.periodic)
    y = forward(params, X, emulate_bf16)["y"].astype(np.float64)
    scale = np.empty(g.nb)
    scale[:g.d * g.nq] = s[0] * cvec[0]
    scale[g.d * g.nq:] = s[1] * cvec[1]
    return (y * scale[None, :]).ravel()


# ---------------------------------------------------------------------------
# training pairs
# ---------------------------------------------------------------------------
def collect_pairs(solver, xstar, ncycles, dtype=np.float64):
    """Plain V-cycles from zero on A x = A x*: after each cycle the residual
    r = b - A x and the kernel-free error e = x* - x."""
    hier = solver.hier
    b = solver.A @ xstar
    x = np.zeros_like(b)
    out = []
    for _ in range(ncycles):
        x = solver.vcycle_unscaled(b, x, dtype)
        r = b - solver.A @ x
        e = hier.project_kernel(xstar - x)
        out.append((r, e))
    return out


def crop(F, shape, periodic, origin, C, halo):
    """Elements origin + [-halo, C + halo)^d of an element field F (NE, ch),
    axis 0 fastest; zero outside non-periodic walls, wrapped on periodic axes."""
    d = len(shape)
    m = C + 2 * halo
    out = np.zeros((m ** d, F.shape[1]))
    for t in range(m ** d):
        c, rem, ok = [], t, True
        for k in range(d):
            v = origin[k] - halo + rem % m
            rem //= m
            if periodic[k]:
                v %= shape[k]
            elif v < 0 or v >= shape[k]:
                ok = False
            c.append(v)
        if ok:
            E = 0
            for k in reversed(range(d)):
                E = E * shape[k] + c[k]
            out[t] = F[E]
    return out


# ---------------------------------------------------------------------------
# guarded outer iteration
# ---------------------------------------------------------------------------
def minres_step(solver, v, z, params, cvec, g, dtype, emulate_bf16=True, minres=True):
    """z + w dx for the V-cycle result z = V(v) (module docstring); also
    returns w.  minres=False: the full step w = 1."""
    Ad = solver.A.astype(dtype)
    d = solver.d
    r2 = (v.astype(dtype) - Ad @ z.astype(dtype)).astype(np.float64)
    dx = correction(params, cvec, g, r2, emulate_bf16)
    if not minres:
        return z + dx, 1.0
    q = (Ad @ dx.astype(dtype)).astype(np.float64)
    den = float(np.dot(d * q, d * q))
    w = float(np.dot(d * r2, d * q)) / den if den > 0 else 0.0
    return z + w * dx, w


def refinement_learned(solver, b, params, cvec, g, tol=1e-10, maxit=50, dtype=np.float32,
                       emulate_bf16=True, minres=True):
    """Iterative refinement x += V(r) + w dx with the guard of the module
    docstring.  Returns x, the residual history and the number of fallback
    events."""
    hier = solver.hier
    b = hier.project_kernel(np.asarray(b, dtype=np.float64))
    bn = np.linalg.norm(b)
    x = np.zeros_like(b)
    hist = [1.0]
    enabled, rho_plain, strikes, events = True, None, 0, 0
    for it in range(maxit):
        r = b - solver.A @ x
        if np.linalg.norm(r) / bn <= tol:
            break
        z = solver.vcycle_unscaled(r, None, dtype)
        use = enabled and it >= 2
        if use:
            x_new = x + minres_step(solver, r, z, params, cvec, g, dtype, emulate_bf16, minres)[0]
        else:
            x_new = x + z
        rel = np.linalg.norm(b - solver.A @ x_new) / bn
        if use:
            ck = rel / hist[-1]
            strikes = strikes + 1 if ck > 1.1 * rho_plain else 0
            if ck > 1.0 or strikes >= 2:
                enabled, events = False, events + 1
                x_new = x + z
                rel = np.linalg.norm(b - solver.A @ x_new) / bn
        x = x_new
        hist.append(rel)
        if it == 1:
            rho_plain = np.sqrt(hist[2] / hist[0])
    return x, np.array(hist), events


def fgmres_learned(solver, b, params, cvec, g, tol=1e-10, m=30, maxit=200, dtype=np.float32, emulate_bf16=True):
    """Flexible GMRES(m), right-preconditioned by z + w dx (module docstring)
    with z = V(v) from zero; modified Gram-Schmidt and Givens rotations in
    FP64 as in the plain FGMRES.  Returns x, the residual history (the Givens
    estimate per iteration, the explicit FP64 residual at each restart) and
    the list of steps w."""
    hier = solver.hier
    b = hier.project_kernel(np.asarray(b, dtype=np.float64))
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    hist = [1.0]
    ws = []
    its = 0
    while its < maxit:
        r = b - solver.A @ x
        beta = np.linalg.norm(r)
        hist[-1] = beta / nb
        if beta / nb <= tol:
            break
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        gv = np.zeros(m + 1)
        gv[0] = beta
        jd = 0
        for j in range(m):
            z = solver.vcycle_unscaled(V[j], None, dtype)
            z, w_ = minres_step(solver, V[j], z, params, cvec, g, dtype, emulate_bf16)
            ws.append(w_)
            Z.append(z)
            w = solver.A @ z
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            V.append(w / H[j + 1, j] if H[j + 1, j] > 0 else w)
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            gv[j + 1] = -sn[j] * gv[j]
            gv[j] = cs[j] * gv[j]
            its += 1
            jd = j + 1
            hist.append(abs(gv[j + 1]) / nb)
            if abs(gv[j + 1]) / nb <= tol or its >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:jd, :jd]), gv[:jd])
        x = x + np.stack(Z[:jd], axis=1) @ y
        hist[-1] = np.linalg.norm(b - solver.A @ x) / nb
        if hist[-1] <= tol:
            break
    return x, np.array(hist), ws
