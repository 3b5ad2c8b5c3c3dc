"""Pins for the warm-start reference: bfloat16 rounding, MLP gradients by
central finite differences, Adam on a quadratic, POD against the SVD."""
import numpy as np

from oracle.learned import adam_step, bf16_round, mlp_forward, mse_loss_grad, pod


def _params(rng, sizes):
    return [((rng.standard_normal((o, i)) / np.sqrt(i)).astype(np.float32),
             (0.1 * rng.standard_normal(o)).astype(np.float32)) for i, o in zip(sizes[:-1], sizes[1:])]


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-9, 3.14159265, -2.5e-3, 65504.0], np.float32)
    r = bf16_round(x)
    # bfloat16 keeps 8 significand bits: 1 + 2^-8 is a tie -> even (1.0);
    # 1 + 3*2^-9 rounds up to 1 + 2^-7
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2**-7
    assert abs(r[3] - 3.140625) < 1e-12
    rel = np.abs(r - x) / np.abs(x)
    assert np.all(rel <= 2**-8 + 1e-12)  # half an ulp of an 8-bit significand


def test_mlp_gradients_finite_difference():
    rng = np.random.default_rng(0)
    sizes = [3, 16, 16, 8, 6]
    P = _params(rng, sizes)
    x = rng.standard_normal((11, 3))
    t = rng.standard_normal((11, 6))
    loss, grads = mse_loss_grad(P, x, t, bf16=False)
    eps = 1e-6
    for l in range(len(P)):
        W, b = P[l]
        for (i, j) in [(0, 0), (W.shape[0] - 1, W.shape[1] - 1), (W.shape[0] // 2, 1)]:
            Wp = W.astype(np.float64).copy()
            Wm = Wp.copy()
            Wp[i, j] += eps
            Wm[i, j] -= eps
            Pp = [(w.astype(np.float64), bb.astype(np.float64)) for w, bb in P]
            Pm = [(w.astype(np.float64), bb.astype(np.float64)) for w, bb in P]
            Pp[l] = (Wp, P[l][1].astype(np.float64))
            Pm[l] = (Wm, P[l][1].astype(np.float64))
            fd = (mse_loss_grad(Pp, x, t, bf16=False)[0] - mse_loss_grad(Pm, x, t, bf16=False)[0]) / (2 * eps)
            assert abs(fd - grads[l][0][i, j]) < 1e-7 * max(1.0, abs(fd)), (l, i, j)
        bp = b.astype(np.float64).copy()
        bm = bp.copy()
        bp[0] += eps
        bm[0] -= eps
        Pp = [(w.astype(np.float64), bb.astype(np.float64)) for w, bb in P]
        Pm = [(w.astype(np.float64), bb.astype(np.float64)) for w, bb in P]
        Pp[l] = (P[l][0].astype(np.float64), bp)
        Pm[l] = (P[l][0].astype(np.float64), bm)
        fd = (mse_loss_grad(Pp, x, t, bf16=False)[0] - mse_loss_grad(Pm, x, t, bf16=False)[0]) / (2 * eps)
        assert abs(fd - grads[l][1][0]) < 1e-7 * max(1.0, abs(fd))


def test_mlp_bf16_close_to_fp():
    rng = np.random.default_rng(1)
    P = _params(rng, [3, 32, 32, 4])
    x = rng.standard_normal((5, 3))
    y1, _ = mlp_forward(P, x, bf16=True)
    y0, _ = mlp_forward(P, x, bf16=False)
    assert np.abs(y1 - y0).max() < 0.05 * np.abs(y0).max()


def test_adam_reduces_loss():
    rng = np.random.default_rng(2)
    P = _params(rng, [3, 32, 32, 2])
    x = rng.uniform(-1, 1, (64, 3))
    t = np.stack([np.sin(2 * x[:, 0]), x[:, 1] * x[:, 2]], 1)
    st = [[(np.zeros_like(W, np.float64), np.zeros_like(W, np.float64)),
           (np.zeros_like(b, np.float64), np.zeros_like(b, np.float64))] for W, b in P]
    l0 = mse_loss_grad(P, x, t)[0]
    for it in range(1, 301):
        _, g = mse_loss_grad(P, x, t)
        P = adam_step(P, g, st, 3e-3, it)
    assert mse_loss_grad(P, x, t)[0] < 0.2 * l0


def test_adam_hand_values():
    """Two Adam steps on one scalar weight and one scalar bias, worked out by
    hand (Kingma and Ba 2015, with the bias corrections 1 - b1^t, 1 - b2^t and
    eps added to the square root of the corrected second moment):
      step 1, g = 0.5:   m = 0.05, v = 0.00025, m^ = 0.5, v^ = 0.25,
                         w -= 0.1 * 0.5 / (0.5 + 1e-8)           -> -0.0999999980
      step 2, g = -0.25: m = 0.045 - 0.025 = 0.02, m^ = 0.02 / 0.19,
                         v = 0.00024975 + 0.0000625 = 0.00031225, v^ = v / 0.001999,
                         w -= 0.1 * 0.1052632 / (0.3952246 + 1e-8) = 0.0266335
    The bias of a tiny gradient g = 1e-9 moves by lr * g / (|g| + eps) =
    lr / 11 on step 1, which fixes where eps enters."""
    W = np.zeros((1, 1), np.float32)
    b = np.zeros(1, np.float32)
    st = [[(np.zeros((1, 1)), np.zeros((1, 1))), (np.zeros(1), np.zeros(1))]]
    P = [(W, b)]
    P = adam_step(P, [(np.full((1, 1), 0.5), np.full(1, 1e-9))], st, 0.1, 1)
    assert abs(P[0][0][0, 0] - (-0.1 * 0.5 / (0.5 + 1e-8))) < 1e-8
    assert abs(P[0][1][0] - (-0.1 / 11.0)) < 1e-8
    w1 = float(P[0][0][0, 0])
    P = adam_step(P, [(np.full((1, 1), -0.25), np.full(1, 0.0))], st, 0.1, 2)
    step2 = 0.1 * (0.02 / 0.19) / (np.sqrt(0.00031225 / 0.001999) + 1e-8)
    assert abs(step2 - 0.0266335) < 1e-6
    assert abs(P[0][0][0, 0] - (w1 - step2)) < 1e-7


def test_pod_matches_svd():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((200, 12)) + 1j * rng.standard_normal((200, 12))
    Phi, sig = pod(X, 5)
    U, S, Vh = np.linalg.svd(X, full_matrices=False)
    assert np.allclose(sig, S[:5], rtol=1e-10)
    assert np.allclose(Phi.conj().T @ Phi, np.eye(5), atol=1e-10)
    # same subspace: projectors agree
    P1 = Phi @ Phi.conj().T
    P2 = U[:, :5] @ U[:, :5].conj().T
    assert np.abs(P1 - P2).max() < 1e-10
