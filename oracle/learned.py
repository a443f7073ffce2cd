"""Learned preconditioner of the masked 2RBT system, in float64: a factorised
approximate inverse P = K^T K whose factor K is a four-layer convolutional
network over the per-sensor slope maps, trained on (residual, exact solution)
pairs, and applied inside flexible preconditioned CG.

The paper leaves preconditioning of its Toeplitz system open (§2.G; the
conclusion names it as the remaining challenge).  This module is the plain
definition of what the library computes for that slot.

Network.  The C = 2 N_gs slope channels of a vector r (W_s^T r: the valid
slopes on the n x n subaperture grid, zeros elsewhere, §2.F) pass through four
linear 3 x 3 convolutions C -> H -> H -> H -> C (H = 32 hidden channels,
zero padding, no bias, no activation):

    h_l[o][y][x] = sum_{i, dy, dx} W_l[o][i][1 + dy][1 + dx] h_{l-1}[i][y + dy][x + dx],

y the grid row, x the column, and K r = W_s h_4 (the valid outputs).  Each
W_l is masked so that K is lower triangular in the order (pixel in row-major
order, then channel): the taps of the next row (dy = +1) and of the next pixel
of the same row (dy = 0, dx = +1) are zero, and the centre tap W_l[o][i][1][1]
is kept only when deg(o) >= deg(i), where input and output channel c has
degree c and hidden channel h degree h mod C (the degree ordering of
autoregressive masks).  Then the diagonal of K is the same at every valid
subaperture, d = diag(D_4 D_3 D_2 D_1) with D_l the masked centre taps, and

    log |det K| = n_vs sum_c log |d_c|.

Preconditioner.  P r = K^T K r (K^T: the adjoint, i.e. the transposed
convolutions in reverse order, between the same restrictions).  P is
symmetric positive definite whenever every d_c != 0.

Training objective.  Kaporin's condition number of the preconditioned matrix
(I. E. Kaporin, Numer. Linear Algebra Appl. 1 (1994)) is
beta(P A) = (tr(P A) / N)^N / det(P A), N = C n_vs.  With P = K^T K,

    log beta = N log(tr(K A K^T) / N) - 2 log |det K| - log det A,

the last term a constant.  For pairs (r, e) with e ~ N(0, I) and r = A e (e is
the exact solution of A e = r), E[(K r) . (K e)] = tr(K A K^T), so the
training objective on a batch of B pairs is

    J = N log(t / N) - 2 n_vs sum_c log |d_c|,   t = (1/B) sum_b (K r_b) . (K e_b).

Minimising beta is the criterion of factorised sparse approximate inverses
(Kolotilina & Yeremin, SIAM J. Matrix Anal. Appl. 14 (1993)); here the factor
is the network.  The optimiser is Adam (Kingma & Ba, ICLR 2015) on FP32 master
weights; the network computes with the master weights rounded to bfloat16
(round to nearest even).

TEST INFRASTRUCTURE ONLY, like the rest of this package.
"""
import numpy as np

from . import geometry as G


# ---------------------------------------------------------------------------
# masks and shapes
# ---------------------------------------------------------------------------

def layer_shapes(C, H=32):
    """(out, in) channels of the four layers."""
    return [(H, C), (H, H), (H, H), (C, H)]


def degrees(C, H=32):
    """Channel degrees of the five activations (input, three hidden, output)."""
    dc = np.arange(C)
    dh = np.arange(H) % C
    return [dc, dh, dh, dh, dc]


def weight_masks(C, H=32):
    """0/1 masks (out, in, 3, 3) of the four layers: no tap on the next row or
    on the next pixel of the same row; the centre tap only from a channel of
    lower or equal degree."""
    deg = degrees(C, H)
    out = []
    for l, (co, ci) in enumerate(layer_shapes(C, H)):
        m = np.ones((co, ci, 3, 3))
        m[:, :, 2, :] = 0.0          # dy = +1
        m[:, :, 1, 2] = 0.0          # dy = 0, dx = +1
        m[:, :, 1, 1] = (deg[l + 1][:, None] >= deg[l][None, :]).astype(float)
        out.append(m)
    return out


def bf16_round(w):
    """Round to the nearest bfloat16 value (ties to even), returned as float64."""
    f = np.asarray(w, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# the network
# ---------------------------------------------------------------------------

def conv3x3(W, h):
    """out[o][y][x] = sum_{i,dy,dx} W[o][i][1+dy][1+dx] h[i][y+dy][x+dx], zero padding."""
    co = W.shape[0]
    ci, n, m = h.shape
    hp = np.zeros((ci, n + 2, m + 2))
    hp[:, 1:-1, 1:-1] = h
    out = np.zeros((co, n, m))
    for ky in range(3):
        for kx in range(3):
            out += np.einsum("oi,iyx->oyx", W[:, :, ky, kx], hp[:, ky:ky + n, kx:kx + m])
    return out


def conv3x3_adjoint(W, g):
    """The adjoint of conv3x3(W, .): h[i][y][x] = sum_{o,dy,dx} W[o][i][1+dy][1+dx] g[o][y-dy][x-dx]."""
    ci = W.shape[1]
    co, n, m = g.shape
    out = np.zeros((ci, n + 2, m + 2))
    for ky in range(3):
        for kx in range(3):
            out[:, ky:ky + n, kx:kx + m] += np.einsum("oi,oyx->iyx", W[:, :, ky, kx], g)
    return out[:, 1:-1, 1:-1]


def conv3x3_weight_grad(h, g):
    """d/dW of sum(g * conv3x3(W, h)): [o][i][ky][kx] = sum_{y,x} g[o][y][x] h[i][y+ky-1][x+kx-1]."""
    ci, n, m = h.shape
    co = g.shape[0]
    hp = np.zeros((ci, n + 2, m + 2))
    hp[:, 1:-1, 1:-1] = h
    out = np.zeros((co, ci, 3, 3))
    for ky in range(3):
        for kx in range(3):
            out[:, :, ky, kx] = np.einsum("oyx,iyx->oi", g, hp[:, ky:ky + n, kx:kx + m])
    return out


def to_maps(v, valid, C):
    """W_s^T: (C n_vs,) valid slopes -> (C, n, n) maps, zeros at invalid subapertures."""
    n = valid.shape[0]
    idx = G.valid_index(valid)
    maps = np.zeros((C, n * n))
    maps[:, idx] = np.asarray(v, dtype=np.float64).reshape(C, idx.size)
    return maps.reshape(C, n, n)


def from_maps(maps, valid):
    """W_s: (C, n, n) maps -> (C n_vs,) values at the valid subapertures."""
    C = maps.shape[0]
    return maps.reshape(C, -1)[:, G.valid_index(valid)].reshape(-1)


def forward_maps(weights, h0):
    """Activations h_0 .. h_4 of the four layers (h0 already on the grid)."""
    hs = [h0]
    for W in weights:
        hs.append(conv3x3(W, hs[-1]))
    return hs


def K_apply(weights, valid, r):
    """K r = W_s h_4, h_0 = W_s^T r."""
    C = weights[-1].shape[0]
    return from_maps(forward_maps(weights, to_maps(r, valid, C))[-1], valid)


def KT_apply(weights, valid, y):
    """K^T y: W_s^T y through the adjoint layers in reverse order, then W_s."""
    C = weights[-1].shape[0]
    g = to_maps(y, valid, C)
    for W in reversed(weights):
        g = conv3x3_adjoint(W, g)
    return from_maps(g, valid)


def precondition(weights, valid, r):
    """z = P r = K^T K r."""
    return KT_apply(weights, valid, K_apply(weights, valid, r))


def centre_diagonal(weights):
    """d = diag(D_4 D_3 D_2 D_1), D_l the centre taps (masks already applied)."""
    D = None
    for W in weights:
        c = W[:, :, 1, 1]
        D = c if D is None else c @ D
    return np.diag(D).copy()


def log_abs_det_K(weights, n_vs):
    return n_vs * float(np.sum(np.log(np.abs(centre_diagonal(weights)))))


def dense_K(weights, valid):
    """K as a dense (N, N) matrix (columns K e_j), for small grids."""
    C = weights[-1].shape[0]
    N = C * int(valid.sum())
    return np.stack([K_apply(weights, valid, np.eye(N)[j]) for j in range(N)], axis=1)


# ---------------------------------------------------------------------------
# training objective, its gradient, one optimiser step
# ---------------------------------------------------------------------------

def objective(weights, valid, R, E):
    """J = N log(t / N) - 2 n_vs sum_c log|d_c|, t = mean_b (K r_b).(K e_b);
    R, E: (B, N) pairs.  Returns (J, t)."""
    n_vs = int(valid.sum())
    C = weights[-1].shape[0]
    N = C * n_vs
    t = float(np.mean([K_apply(weights, valid, r) @ K_apply(weights, valid, e) for r, e in zip(R, E)]))
    return N * np.log(t / N) - 2.0 * log_abs_det_K(weights, n_vs), t


def kaporin_dense(weights, valid, A):
    """log of Kaporin's condition number of P A, P = K^T K, from dense matrices."""
    K = dense_K(weights, valid)
    M = K @ A @ K.T
    N = A.shape[0]
    return N * np.log(np.trace(M) / N) - np.linalg.slogdet(M)[1]


def objective_grad(weights, valid, R, E, masks):
    """dJ/dW_l by back-propagation through the linear layers, plus the
    log-determinant term; masked like the weights.  Returns (grads, J, t)."""
    n_vs = int(valid.sum())
    C = weights[-1].shape[0]
    N = C * n_vs
    B = len(R)
    vmask = np.asarray(valid, dtype=float)[None]
    acts_r = [forward_maps(weights, to_maps(r, valid, C)) for r in R]
    acts_e = [forward_maps(weights, to_maps(e, valid, C)) for e in E]
    t = float(np.mean([np.sum(a[-1] * vmask * b[-1]) for a, b in zip(acts_r, acts_e)]))
    J = N * np.log(t / N) - 2.0 * log_abs_det_K(weights, n_vs)
    grads = [np.zeros_like(W) for W in weights]
    scale = N / t / B
    for a, b in zip(acts_r, acts_e):
        for acts, other in ((a, b), (b, a)):
            g = scale * vmask * other[-1]          # dJ/d(output maps) of this branch
            for l in range(3, -1, -1):
                grads[l] += conv3x3_weight_grad(acts[l], g)
                g = conv3x3_adjoint(weights[l], g)
    # - 2 n_vs sum_c log|d_c|: d/dD_l = (D_4..D_{l+1})^T diag(1/d) (D_{l-1}..D_1)^T
    Ds = [W[:, :, 1, 1] for W in weights]
    d = centre_diagonal(weights)
    for l in range(4):
        above = np.eye(Ds[l].shape[0])
        for k in range(l + 1, 4):
            above = Ds[k] @ above
        below = np.eye(Ds[0].shape[1])
        for k in range(l):
            below = Ds[k] @ below
        grads[l][:, :, 1, 1] += -2.0 * n_vs * (above.T @ np.diag(1.0 / d) @ below.T)
    return [g * m for g, m in zip(grads, masks)], J, t


def adam_step(w, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) of the arrays in place;
    step counts from 1.  Returns (w, m, v)."""
    m[...] = beta1 * m + (1.0 - beta1) * g
    v[...] = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    w[...] = w - lr * mh / (np.sqrt(vh) + eps)
    return w, m, v


def train_step(master, adam_m, adam_v, step, valid, R, E, masks, lr):
    """One training step as the library takes it: the gradient at the
    bfloat16-rounded master weights, Adam on the master weights.  Arrays are
    updated in place; returns (J, t) at the weights used."""
    used = [bf16_round(w) * m for w, m in zip(master, masks)]
    grads, J, t = objective_grad(used, valid, R, E, masks)
    for w, g, m_, v_ in zip(master, grads, adam_m, adam_v):
        adam_step(w, g, m_, v_, step, lr)
    for w, m in zip(master, masks):
        w *= m
    return J, t
