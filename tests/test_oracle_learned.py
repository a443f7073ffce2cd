"""Pins of the learned-preconditioner oracle (oracle/learned.py) and of flexible
PCG (oracle/solve.fpcg): each check is independent of the code it pins
(library routines, exact identities, finite differences, closed forms)."""
import numpy as np
import pytest
import scipy.signal

import workloads as W
from oracle import learned as Lr
from oracle.covariance import system_matrix
from oracle.solve import cg, cholesky_solve, fpcg, pcg


def _weights(C, H, seed, masks=None, identity=0.0):
    rng = np.random.default_rng(seed)
    masks = masks or Lr.weight_masks(C, H)
    ws = []
    for (co, ci), m in zip(Lr.layer_shapes(C, H), masks):
        w = rng.standard_normal((co, ci, 3, 3)) / np.sqrt(9 * ci)
        if identity:
            w[:, :, 1, 1] += identity * (np.arange(co)[:, None] % C == np.arange(ci)[None, :] % C)
        ws.append(w * m)
    return ws


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    Wt = rng.standard_normal((3, 2, 3, 3))
    h = rng.standard_normal((2, 5, 7))
    out = Lr.conv3x3(Wt, h)
    for o in range(3):
        ref = sum(scipy.signal.correlate2d(h[i], Wt[o, i], mode="same", boundary="fill") for i in range(2))
        np.testing.assert_allclose(out[o], ref, rtol=1e-13, atol=1e-13)


def test_conv_adjoint_identity_and_weight_grad():
    rng = np.random.default_rng(1)
    Wt = rng.standard_normal((4, 3, 3, 3))
    h = rng.standard_normal((3, 6, 5))
    g = rng.standard_normal((4, 6, 5))
    lhs = np.sum(Lr.conv3x3(Wt, h) * g)
    rhs = np.sum(h * Lr.conv3x3_adjoint(Wt, g))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # sum(g * conv(W, h)) is linear in W: its gradient is exact under any finite step
    G = Lr.conv3x3_weight_grad(h, g)
    D = rng.standard_normal(Wt.shape)
    f = lambda w: np.sum(g * Lr.conv3x3(w, h))
    assert abs((f(Wt + D) - f(Wt)) - np.sum(G * D)) < 1e-11 * abs(np.sum(G * D))


def test_masks_make_K_triangular_and_logdet_exact():
    wl = W.tiny(n=5, n_gs=2, seed=3)
    C, H = 2 * wl.n_gs, 8
    ws = _weights(C, H, 4, identity=1.0)
    K = Lr.dense_K(ws, wl.valid)
    nv = int(wl.valid.sum())
    # reorder (channel, valid pixel) -> (valid pixel, channel): lower triangular
    perm = np.array([c * nv + v for v in range(nv) for c in range(C)])
    Kp = K[np.ix_(perm, perm)]
    assert np.abs(np.triu(Kp, 1)).max() == 0.0
    sign, logdet = np.linalg.slogdet(K)
    assert sign != 0
    assert abs(logdet - Lr.log_abs_det_K(ws, nv)) < 1e-10 * max(1.0, abs(logdet))
    # the diagonal of K is d at every valid subaperture
    d = Lr.centre_diagonal(ws)
    np.testing.assert_allclose(np.diag(Kp), np.tile(d, nv), rtol=1e-12)


def test_unmasked_taps_break_triangularity():
    """A plausible slip (the next-pixel tap left in) is caught by the triangular check."""
    wl = W.tiny(n=4, n_gs=1, seed=5)
    C, H = 2, 4
    masks = Lr.weight_masks(C, H)
    masks[1][:, :, 1, 2] = 1.0
    ws = _weights(C, H, 6, masks=masks, identity=1.0)
    K = Lr.dense_K(ws, wl.valid)
    nv = int(wl.valid.sum())
    perm = np.array([c * nv + v for v in range(nv) for c in range(C)])
    assert np.abs(np.triu(K[np.ix_(perm, perm)], 1)).max() > 0.0


def test_preconditioner_is_KtK_and_spd():
    wl = W.tiny(n=5, n_gs=2, seed=7)
    C, H = 2 * wl.n_gs, 8
    ws = _weights(C, H, 8, identity=1.0)
    K = Lr.dense_K(ws, wl.valid)
    N = K.shape[0]
    P = np.stack([Lr.precondition(ws, wl.valid, np.eye(N)[j]) for j in range(N)], axis=1)
    np.testing.assert_allclose(P, K.T @ K, rtol=1e-11, atol=1e-12 * np.abs(P).max())
    assert np.allclose(P, P.T, atol=1e-12 * np.abs(P).max())
    assert np.linalg.eigvalsh(0.5 * (P + P.T)).min() > 0


def test_kaporin_identity_and_unbiased_trace():
    wl = W.tiny(n=4, n_gs=2, seed=9)
    C, H = 2 * wl.n_gs, 8
    ws = _weights(C, H, 10, identity=1.0)
    A = system_matrix(wl)
    K = Lr.dense_K(ws, wl.valid)
    lam = np.linalg.eigvalsh(K @ A @ K.T)
    N = A.shape[0]
    beta_eig = N * np.log(lam.mean()) - np.sum(np.log(lam))
    assert abs(Lr.kaporin_dense(ws, wl.valid, A) - beta_eig) < 1e-9 * abs(beta_eig)
    # the pair estimator: E[(K A e).(K e)] = tr(K A K^T) for e ~ N(0, I)
    rng = np.random.default_rng(11)
    E = rng.standard_normal((4000, N))
    R = E @ A
    KE, KR = E @ K.T, R @ K.T
    samples = np.sum(KE * KR, axis=1)
    tr = np.trace(K @ A @ K.T)
    assert abs(samples.mean() - tr) < 4 * samples.std() / np.sqrt(len(samples))
    # the training objective with those pairs = Kaporin's number + log det A, to sampling error
    J, t = Lr.objective(ws, wl.valid, R[:50], E[:50])
    np.testing.assert_allclose(t, samples[:50].mean(), rtol=1e-12)


def test_objective_gradient_by_central_differences():
    wl = W.tiny(n=4, n_gs=1, seed=12)
    C, H = 2 * wl.n_gs, 4
    masks = Lr.weight_masks(C, H)
    ws = _weights(C, H, 13, masks=masks, identity=1.0)
    A = system_matrix(wl)
    rng = np.random.default_rng(14)
    E = rng.standard_normal((3, A.shape[0]))
    R = E @ A
    grads, J, t = Lr.objective_grad(ws, wl.valid, R, E, masks)
    J0, _ = Lr.objective(ws, wl.valid, R, E)
    assert abs(J - J0) < 1e-10 * abs(J0)
    h = 1e-6
    checked = 0
    for l in range(4):
        for (o, i, ky, kx) in [(0, 0, 1, 1), (1, 0, 0, 2), (0, 1, 1, 0), (1, 1, 1, 1), (0, 0, 0, 0)]:
            if o >= ws[l].shape[0] or i >= ws[l].shape[1] or masks[l][o, i, ky, kx] == 0:
                continue
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[l][o, i, ky, kx] += h
            wm[l][o, i, ky, kx] -= h
            fd = (Lr.objective(wp, wl.valid, R, E)[0] - Lr.objective(wm, wl.valid, R, E)[0]) / (2 * h)
            assert abs(fd - grads[l][o, i, ky, kx]) < 1e-5 * max(1.0, abs(fd)), (l, o, i, ky, kx)
            checked += 1
    assert checked >= 12
    for g, m in zip(grads, masks):
        assert np.all(g[m == 0] == 0)


def test_adam_closed_form_first_two_steps():
    g1 = np.array([0.5, -2.0, 1e-3])
    g2 = np.array([-1.0, 1.0, 2e-3])
    w = np.array([1.0, 2.0, 3.0])
    m = np.zeros(3)
    v = np.zeros(3)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    Lr.adam_step(w, g1, m, v, 1, lr)
    np.testing.assert_allclose(w, [1.0, 2.0, 3.0] - lr * g1 / (np.abs(g1) + eps), rtol=1e-14)
    w1 = w.copy()
    Lr.adam_step(w, g2, m, v, 2, lr)
    m2 = b1 * (1 - b1) * g1 + (1 - b1) * g2
    v2 = b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2
    np.testing.assert_allclose(w, w1 - lr * (m2 / (1 - b1 ** 2)) / (np.sqrt(v2 / (1 - b2 ** 2)) + eps), rtol=1e-14)


def test_bf16_round_matches_torch():
    import torch
    rng = np.random.default_rng(15)
    x = rng.standard_normal(10000) * 10.0 ** rng.uniform(-5, 5, 10000)
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(Lr.bf16_round(x), ref)
    # ties to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert Lr.bf16_round(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert Lr.bf16_round(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6


def test_fpcg_reduces_to_cg_and_pcg():
    """Polak-Ribiere beta equals Fletcher-Reeves when r'.u = 0, which CG keeps to
    rounding: on a well-conditioned system the iterates agree to rounding; on the
    10x10 workload (condition 8.9e3) over the first iterations, before the loss of
    orthogonality separates the two forms."""
    rng = np.random.default_rng(16)
    Q, _ = np.linalg.qr(rng.standard_normal((200, 200)))
    B = Q @ np.diag(np.linspace(1.0, 10.0, 200)) @ Q.T
    b = rng.standard_normal(200)
    Bf = lambda x: B @ x
    x1, it1 = cg(Bf, b, tol=1e-14, maxiter=20)
    x2, it2 = fpcg(Bf, lambda r: r.copy(), b, tol=1e-14, maxiter=20)
    assert it1 == it2 == 20
    assert np.linalg.norm(x1 - x2) < 1e-13 * np.linalg.norm(x1)
    Pm = Q @ np.diag(np.linspace(0.5, 2.0, 200)[::-1]) @ Q.T
    x3, _ = pcg(Bf, lambda r: Pm @ r, b, tol=1e-14, maxiter=15)
    x4, _ = fpcg(Bf, lambda r: Pm @ r, b, tol=1e-14, maxiter=15)
    assert np.linalg.norm(x3 - x4) < 1e-13 * np.linalg.norm(x3)
    wl = W.lgs3_10x10()
    A = system_matrix(wl)
    s = W.turbulent_slopes(wl)[0].astype(np.float64)
    x5, _ = cg(lambda x: A @ x, s, tol=1e-14, maxiter=6)
    x6, _ = fpcg(lambda x: A @ x, lambda r: r.copy(), s, tol=1e-14, maxiter=6)
    assert np.linalg.norm(x5 - x6) < 1e-12 * np.linalg.norm(x5)


def test_fpcg_falls_back_to_cg_and_converges():
    wl = W.lgs3_10x10()
    A = system_matrix(wl)
    s = W.turbulent_slopes(wl)[0].astype(np.float64)
    xref = cholesky_solve(A, s)
    # a preconditioner that is not positive: plain CG takes over
    x, it, hist, fb = fpcg(lambda v: A @ v, lambda r: -r, s, tol=1e-10, maxiter=5000, history=True)
    assert fb
    assert np.linalg.norm(x - xref) < 1e-7 * np.linalg.norm(xref)
    # the learned preconditioner with generic weights: SPD, converges to the Cholesky solution
    C = 2 * wl.n_gs
    ws = _weights(C, 32, 17, identity=1.0)
    x, it, hist, fb = fpcg(lambda v: A @ v, lambda r: Lr.precondition(ws, wl.valid, r), s, tol=1e-10,
                           maxiter=5000, history=True)
    assert not fb
    assert np.linalg.norm(x - xref) < 1e-7 * np.linalg.norm(xref)


@pytest.mark.slow
def test_training_steps_lower_the_kaporin_number():
    """A few oracle training steps on a tiny system lower the exact (dense)
    Kaporin number: the objective's gradient points the right way."""
    wl = W.tiny(n=4, n_gs=1, seed=18)
    C, H = 2 * wl.n_gs, 8
    masks = Lr.weight_masks(C, H)
    master = _weights(C, H, 19, masks=masks, identity=1.0)
    A = system_matrix(wl)
    rng = np.random.default_rng(20)
    E = rng.standard_normal((64, A.shape[0]))
    R = E @ A
    ms = [np.zeros_like(w) for w in master]
    vs = [np.zeros_like(w) for w in master]
    k0 = Lr.kaporin_dense([Lr.bf16_round(w) for w in master], wl.valid, A)
    for step in range(1, 41):
        idx = rng.integers(0, 64, 16)
        Lr.train_step(master, ms, vs, step, wl.valid, R[idx], E[idx], masks, 1e-2)
    k1 = Lr.kaporin_dense([Lr.bf16_round(w) for w in master], wl.valid, A)
    assert k1 < k0
