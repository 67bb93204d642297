"""The exact sPAM states and the surrogate of Sec. 4.3 through the C ABI:
vine_spam_solve against the FP64 oracle's inverse of Eq. 1 (saturated and unsaturated
states, zero, negative and beyond-slack strains), vine_mlp_forward against the network
written out in numpy, and a short training on GPU-solved states that reaches the paper's
error scale."""
import numpy as np
import pytest

from oracle import synthesis as S

pytestmark = pytest.mark.gpu


def test_spam_states_match_the_oracle():
    from paper_2509_15180_amd import vinesim as V
    rng = np.random.default_rng(7)
    l0 = np.concatenate([rng.uniform(0.02, 0.08, 40), [0.02, 0.04, 0.08, 0.05, 0.03, 0.06]])
    eps = np.concatenate([rng.uniform(0.0, 0.3, 40), [0.0, -0.01, 5.0, 0.2, 0.4199, 0.12]])
    import time
    V.spam_solve(eps[:1], l0[:1])  # load the kernels
    t0 = time.perf_counter()
    got = V.spam_solve(eps, l0)
    t_gpu = time.perf_counter() - t0
    worst = 0.0
    t0 = time.perf_counter()
    ref = [S.spam_inverse(float(eps[i]), float(l0[i])) for i in range(len(eps))]
    t_ref = time.perf_counter() - t0
    print(f"{len(eps)} exact states: {t_gpu * 1e3:.2f} ms on the GPU (one call), "
          f"{t_ref * 1e3:.0f} ms with the oracle (one thread)", flush=True)
    for i in range(len(eps)):
        m, phi, G = ref[i]
        assert abs(got[i, 0] - m) <= 1e-13, i
        assert abs(got[i, 1] - phi) <= 1e-11, i
        assert abs(got[i, 2] - G) <= 1e-11 * max(G, 1e-6), i
        worst = max(worst, abs(got[i, 0] - m))
    slack = eps >= 5.0
    assert np.all(got[slack, 0] == 0.5) and np.all(got[slack, 2] == 0.0)
    print(f"sPAM states: {len(eps)} against the oracle, max |dm| {worst:.1e}", flush=True)


def test_surrogate_forward_is_the_network():
    from paper_2509_15180_amd import surrogate as SG
    from paper_2509_15180_amd import vinesim as V
    rng = np.random.default_rng(8)
    w = rng.normal(0.0, 1.0, 162)
    x = rng.uniform(-1.0, 2.0, (5000, 2))
    y = V.mlp_forward(w, x)
    W1, b1, W2, b2 = w[:64].reshape(32, 2), w[64:96], w[96:160].reshape(2, 32), w[160:]
    ref = np.array([[b2[o] + sum(W2[o, k] * max(W1[k, 0] * xi[0] + W1[k, 1] * xi[1] + b1[k], 0.0)
                                 for k in range(32)) for o in range(2)] for xi in x[:200]])
    assert np.abs(y[:200] - ref).max() <= 1e-12
    assert np.abs(y - SG.forward(w, x)).max() <= 1e-12


def test_short_training_reaches_the_error_scale():
    from paper_2509_15180_amd import surrogate as SG
    from paper_2509_15180_amd import vinesim as V
    D = SG.samples(6000, seed=3)
    X = SG.scale_in(D[:, 0], D[:, 1])
    Y = np.column_stack([D[:, 2] / 0.5, D[:, 3] / (np.pi / 2)])
    w, hist = SG.train(X[:5000], Y[:5000], X[5000:5500], Y[5000:5500], epochs=60, seed=3)
    mse = float(np.mean((V.mlp_forward(w, X[5500:]) - Y[5500:]) ** 2))
    print(f"surrogate after 60 epochs on 5000 states: test MSE {mse:.2e}", flush=True)
    assert mse <= 0.01
