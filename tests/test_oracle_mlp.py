"""Pins of the sizing network oracle: finite differences and Adam closed forms."""
import numpy as np

from oracle import mlp


def test_param_count():
    assert mlp.n_params() == 64 * 32 + 64 + 64 * 64 + 64 + 2 * 64 + 2


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    th = rng.standard_normal(mlp.n_params()) * 0.2
    X = rng.standard_normal((7, 32))
    T = rng.standard_normal((7, 2))
    g = mlp.grad(th, X, T)
    idx = rng.choice(th.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (mlp.loss(th + e, X, T) - mlp.loss(th - e, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9


def test_forward_is_relu_mlp_by_hand():
    """A 1-sample forward against a hand-expanded two-hidden-layer formula."""
    rng = np.random.default_rng(1)
    th = rng.standard_normal(mlp.n_params())
    x = rng.standard_normal(32)
    (W1, b1), (W2, b2), (W3, b3) = mlp.unpack(th)
    h1 = [max(0.0, sum(W1[o, i] * x[i] for i in range(32)) + b1[o]) for o in range(64)]
    h2 = [max(0.0, sum(W2[o, i] * h1[i] for i in range(64)) + b2[o]) for o in range(64)]
    y = [sum(W3[o, i] * h2[i] for i in range(64)) + b3[o] for o in range(2)]
    out, _ = mlp.forward(th, x[None, :])
    assert np.allclose(out[0], y, rtol=1e-12, atol=1e-12)


def test_adam_first_step_is_signed_lr():
    """First Adam step: m-hat = g, v-hat = g^2, so the update is lr g/(|g|+eps)."""
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_training_reduces_loss():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((64, 32))
    T = np.stack([np.tanh(X[:, 0]), X[:, 1] * 0.5], axis=1)
    th = rng.standard_normal(mlp.n_params()) * 0.1
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    l0 = mlp.loss(th, X, T)
    for s in range(1, 201):
        th, m, v = mlp.adam_step(th, mlp.grad(th, X, T), m, v, s, 3e-3)
    assert mlp.loss(th, X, T) < 0.2 * l0


# ------------------------------------------------------- sizing features ---
def test_probe_features_scale_invariant_and_rank_revealing():
    """Both halves are log10 ratios: unchanged by scaling G.  The probe half
    (s_2, s_4, ..., s_16 over s_1) is non-increasing; a rank-r matrix
    (r < 16) shows a drop to the floor after its r-th singular value in the
    probe and after its r-th sketch column in the profile (the sketch has
    rank r, so later columns lie in the span of the first r)."""
    from oracle.sizing import features
    rng = np.random.default_rng(3)
    m, n, r = 300, 120, 6
    G1 = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    G2 = rng.standard_normal((250, n))
    k, cap = 8, 120                      # grid {12, 16, 24, 40}: L = 40, profile at 2, 4, 6, 8, 12, 16, 24, 40
    f = features(G1, G2, 9, k, cap)
    f2 = features(7.5 * G1, 0.01 * G2, 9, k, cap)
    assert f.shape == (32,)
    live = f > -8                        # entries above the floor
    assert np.array_equal(live, f2 > -8)
    assert np.allclose(f[live], f2[live], atol=1e-12)
    assert np.all(np.diff(f[:8]) <= 1e-12) and np.all(np.diff(f[16:24]) <= 1e-12)
    assert np.all(f[:3] > -3) and np.all(f[3:8] == -8.0)        # probe: s_2, s_4, s_6 live, s_8.. floor
    assert np.all(f[8:11] > -3) and np.all(f[11:16] == -8.0)    # profile: columns 2, 4, 6 live, 8.. floor
    assert np.all(f[16:] > -3)                                   # full-rank Gaussian G2


def test_sketch_profile_is_distance_to_previous_columns():
    """rho_j is the distance of sketch column j from the span of columns
    1..j-1: brute force by least squares on each prefix."""
    from oracle.philox import gaussian_matrix
    from oracle.sizing import sketch_profile
    rng = np.random.default_rng(5)
    G = rng.standard_normal((90, 40)) * (0.8 ** np.arange(40))[None, :]
    L = 12
    rho = sketch_profile(G, 6, 2, L)
    S = G @ gaussian_matrix(6, 2, 40, 0, L)
    ref = [np.linalg.norm(S[:, 0])]
    for j in range(1, L):
        c, *_ = np.linalg.lstsq(S[:, :j], S[:, j], rcond=None)
        ref.append(np.linalg.norm(S[:, j] - S[:, :j] @ c))
    assert np.allclose(rho, ref, rtol=1e-10)


def test_profile_positions():
    from oracle.sizing import profile_positions
    assert profile_positions(20, 52) == [5, 10, 15, 20, 24, 28, 36, 52]
    assert profile_positions(200, 224) == [50, 100, 150, 200, 204, 208, 216, 224]
    assert profile_positions(3, 6) == [1, 2, 3, 3, 6, 6, 6, 6]
    assert profile_positions(1, 2) == [1, 1, 1, 1, 2, 2, 2, 2]


def test_probe_spectrum_of_orthonormal_rows_is_gaussian_block():
    """For G with orthonormal rows spanning R^n (G = I_n), G Omega16 is the
    Gaussian block itself, so the probe spectrum equals its singular values."""
    from oracle.philox import gaussian_matrix
    from oracle.sizing import probe_spectrum
    n = 64
    s = probe_spectrum(np.eye(n), 4, 1)
    ref = np.linalg.svd(gaussian_matrix(4, 1, n, 0, 16), compute_uv=False)
    assert np.allclose(s, ref, rtol=1e-13)


def test_decide_rounds_up_to_grid():
    from oracle.sizing import decide, l_grid
    assert l_grid(20, 1000) == [24, 28, 36, 40, 52]
    assert decide([0.0, 0.0], 20, 1000) == (24, 0)
    assert decide([np.log2(30 / 20), 1.3], 20, 1000) == (36, 2)
    assert decide([5.0, 9.0], 20, 1000) == (52, 3)
    assert decide([0.5, -2.0], 20, 30) == (30, 0)
    # q rounds up from y1 = 0.1 on
    assert decide([0.0, 0.09], 20, 1000)[1] == 0 and decide([0.0, 0.1], 20, 1000)[1] == 1
    assert decide([0.0, 1.09], 20, 1000)[1] == 1 and decide([0.0, 1.1], 20, 1000)[1] == 2
