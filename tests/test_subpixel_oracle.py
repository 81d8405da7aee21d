"""Pins for the subpixel oracle (oracle/subpixel.py).  CPU only."""
import numpy as np
import pytest

from oracle import subpixel as S

F32 = np.float32


def test_bf16_rounding_matches_torch_and_ties_to_even():
    import torch

    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 10, 5000), rng.normal(0, 1e-3, 1000),
                        [1.0, 1 + 2 ** -8, 1 + 2 ** -8 + 2 ** -20, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 0.0]]).astype(F32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(S.bf16(x), want)
    # halfway cases go to the even neighbour
    assert S.bf16(np.array([1 + 2 ** -8], F32))[0] == 1.0
    assert S.bf16(np.array([1 + 3 * 2 ** -8], F32))[0] == F32(1 + 2 ** -6)


def test_param_count():
    assert S.N_PARAMS == 5954


def test_backward_matches_finite_differences():
    """float64 definitions: analytic gradient vs central differences."""
    rng = np.random.default_rng(2)
    theta = S.init_params(3).astype(np.float64) + rng.normal(0, 0.05, S.N_PARAMS)
    patches = rng.normal(20, 40, size=(6, 5, 5))
    target = rng.uniform(-0.5, 0.5, size=(6, 2))
    g, _ = S.mlp_backward(theta, patches, target, bf16_ops=False)
    idx = rng.choice(S.N_PARAMS, size=120, replace=False)
    idx = np.concatenate([idx, np.arange(S.N_PARAMS - 130, S.N_PARAMS)])  # all of W3, b3
    h = 1e-6
    for i in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        lp = S.mlp_loss(S.mlp_forward(tp, patches, bf16_ops=False)[0], target)
        lm = S.mlp_loss(S.mlp_forward(tm, patches, bf16_ops=False)[0], target)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_forward_hand_built_network():
    """W1 copies pixels (2,2) and (2,3) into hidden units 0 and 1, W2 passes
    them through, W3 outputs (h0 - h1, 2*h1) + b3."""
    p = {name: np.zeros(shape, np.float64) for name, shape in S.SHAPES}
    p["W1"][12, 0] = 1.0
    p["W1"][13, 1] = 1.0
    p["W2"][0, 0] = 1.0
    p["W2"][1, 1] = 1.0
    p["W3"][0, 0] = 1.0
    p["W3"][1, 0] = -1.0
    p["W3"][1, 1] = 2.0
    p["b3"][:] = [0.25, -0.5]
    theta = S.pack(p)
    patch = np.zeros((2, 5, 5))
    patch[0, 2, 2], patch[0, 2, 3] = 150.0, 75.0
    patch[1, 2, 2], patch[1, 2, 3] = -30.0, 300.0      # ReLU zeroes the first unit
    y, _ = S.mlp_forward(theta, patch, photon_adu=150.0, bf16_ops=False)
    assert np.allclose(y, [[1.0 - 0.5 + 0.25, 1.0 - 0.5], [0.0 - 2.0 + 0.25, 4.0 - 0.5]])
    yb, _ = S.mlp_forward(theta.astype(F32), patch, photon_adu=150.0, bf16_ops=True)
    assert np.allclose(yb, y, atol=1e-2)


def test_adam_first_step_is_signed_lr():
    theta = np.zeros(10, F32)
    g = np.linspace(-1, 1, 10).astype(F32)
    g[4] = 0.0
    t, m, v = S.adam(theta, np.zeros(10, F32), np.zeros(10, F32), g, 1, 1e-3)
    exp = -1e-3 * np.sign(g)
    assert np.allclose(t, exp, atol=1e-9)


@pytest.mark.parametrize("t_nb", [9.0, 0.0])
def test_centroid_closed_forms(t_nb):
    P = np.zeros((5, 5, 5), F32)
    P[0, 2, 2] = 100                                  # single pixel -> 0, 0
    P[1, 2, 2], P[1, 2, 3] = 60, 40                   # split in x -> dx = 0.4
    P[2, 1, 2], P[2, 2, 2], P[2, 3, 2] = 30, 60, 30   # symmetric in y -> 0
    P[3, 2, 2], P[3, 3, 1] = 50, 50                   # diagonal -> (0.5, -0.5)
    P[4, 2, 2], P[4, 2, 1], P[4, 0, 0] = 80, -20, 500  # negative and outside-3x3 pixels ignored
    c = S.centroid(P, t_nb)
    assert np.allclose(c, [[0, 0], [0, 0.4], [0, 0], [0.5, -0.5], [0, 0]], atol=1e-7)
    # the neighbour threshold is strict
    Q = np.zeros((1, 5, 5), F32)
    Q[0, 2, 2], Q[0, 2, 3] = 50, 9.0
    assert S.centroid(Q, 9.0)[0, 1] == 0.0
    assert S.centroid(Q, 8.0)[0, 1] == F32(9.0 / 59.0)


def test_eta_maps_uniform_to_identity():
    rng = np.random.default_rng(4)
    c = rng.uniform(-0.5, 0.5, size=(200000, 2))
    tab = S.eta_table(c, nbins=511)
    q = np.linspace(-0.45, 0.45, 19)
    out = S.eta_apply(np.stack([q, q], axis=1), tab)
    assert np.allclose(out, np.stack([q, q], axis=1), atol=0.01)
    # monotone mapping of a skewed distribution onto uniform positions
    s = np.tanh(rng.uniform(-2, 2, size=(100000, 2))) * 0.5
    tab2 = S.eta_table(s, nbins=512)
    u = S.eta_apply(s, tab2)
    hist = np.histogram(u[:, 0], bins=10, range=(-0.5, 0.5))[0]
    assert hist.min() > 0.9 * len(s) / 10


def test_eta_table_hand_count():
    """4 centroids, 4 bins of width 0.5 on [-1, 1]: x-coordinates -0.5, 0, 0,
    0.5 fall in bins 1, 2, 2, 3 (a coordinate on an edge belongs to the bin
    above it); y-coordinates -1, 1, 1, 0.99 in bins 0, 3, 3, 3 (1 is in the
    last bin)."""
    c = np.array([[-1.0, -0.5], [1.0, 0.0], [1.0, 0.0], [0.99, 0.5]], F32)
    tab = S.eta_table(c, nbins=4)
    assert np.array_equal(tab[1], np.array([0, 0, 0.25, 0.75, 1.0], F32))
    assert np.array_equal(tab[0], np.array([0, 0.25, 0.25, 0.25, 1.0], F32))
    # CDF at the x edges -0.5 and 0 -> positions -0.25 and 0.25 - 0.5
    out = S.eta_apply(np.array([[0.0, -0.5], [0.0, 0.0], [0.0, 0.25]], F32), tab)
    assert np.allclose(out[:, 1], [0.0 - 0.5, 0.25 - 0.5, 0.5 * (0.25 + 0.75) - 0.5])
