"""The training recipe's gradient histories and the input-range bound the
hybrid gate takes from them (train.input_quantile), on the CPU.

The stationary Ornstein-Uhlenbeck entries a, b, c of a box are N(0, sd^2)
and the gradient [[a, b, 0], [c, -a, 0], 0] has squared Frobenius norm
2 a^2 + b^2 + c^2; the bound is checked against an independent Monte
Carlo sample of that law (other generator, 10^6 draws)."""
import numpy as np

from paper_2512_13267_amd import train


def test_ou_histories_are_stationary_with_the_set_amplitude():
    G = train.ou_gradients(4000, 60, sd=0.07, corr=5.0, seed=3)
    a, b, c, d = G[:, :, 0], G[:, :, 1], G[:, :, 3], G[:, :, 4]
    assert np.array_equal(d, -a)
    assert np.all(G[:, :, [2, 5, 6, 7, 8]] == 0.0)
    for x in (a, b, c):
        for t in (0, 30, 59):
            assert abs(x[t].std() / 0.07 - 1.0) < 0.05
    # lag-1 correlation exp(-1/corr)
    r = np.mean(a[1:] * a[:-1]) / np.mean(a * a)
    assert abs(r - np.exp(-1.0 / 5.0)) < 0.02


def test_input_quantile_matches_the_frobenius_law():
    sd = train.GRAD_SD
    q = train.input_quantile(0.9, 3000, train.HIST + 40, seed_k=17, amp_range=(0.0, 0.0), corr_range=(1.0, 1.0))
    rng = np.random.default_rng(12345)
    x = rng.normal(size=(1_000_000, 3)) * sd
    ref = np.quantile(np.sqrt(2.0 * x[:, 0] ** 2 + x[:, 1] ** 2 + x[:, 2] ** 2), 0.9)
    assert abs(q / ref - 1.0) < 0.01, (q, ref)
    # the diagonal counted once would give a visibly smaller bound
    wrong = np.quantile(np.sqrt(x[:, 0] ** 2 + x[:, 1] ** 2 + x[:, 2] ** 2), 0.9)
    assert abs(wrong / ref - 1.0) > 0.05


def test_shear_recipe_adds_only_to_the_xy_entry():
    _, G0, _, _, _ = train.gradient_histories(64, 50, seed_k=5)
    _, G1, _, _, sh = train.gradient_histories(64, 50, seed_k=5, shear=(0.5, 0.0, 0.5))
    diff = G1 - G0
    assert np.all(diff[:, :, [0, 2, 3, 4, 5, 6, 7, 8]] == 0.0)
    moved = np.abs(diff[:, :, 1]).max(axis=0) > 0
    assert np.array_equal(moved, sh > 0) and 0 < moved.sum() < 64
