"""The packaged trained surrogate on fresh micro-DPD data (seeds never used
in training), against the methods without it.

A single interval-averaged stress target carries DPD noise of the order of
its own size, so the comparison uses targets averaged over 8 replicas
(same start and gradients, different random-force streams), whose noise is
sqrt(8) smaller.  Against those the ensemble mean must beat
  * no learned model (a zero prediction, what the macro side would get
    without a stress model: relative L2 = 1) and the same architecture
    untrained, by far;
  * the linear closure of the current gradient alone (a Newtonian-like map
    with intercept, fitted by least squares on a separate fresh data set):
    the history of the gradient is what the network adds.
The replicas' own scatter gives the noise left in the 8-replica mean; the
ensemble's error may not exceed it by much (the network predicts the
noise-free mean).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

R = 8


def _replica_means(X, T, box_id, step_id):
    """Rows grouped by (unique box, step) with all R replicas present: the
    shared features, the replica-mean target and the mean squared deviation
    of the replicas from it (the noise of one target)."""
    b = box_id.cpu().numpy() // R
    s = step_id.cpu().numpy()
    key = b.astype(np.int64) * 100000 + s
    order = np.argsort(key, kind="stable")
    key = key[order]
    starts = np.flatnonzero(np.r_[True, key[1:] != key[:-1]])
    counts = np.diff(np.r_[starts, key.size])
    full = starts[counts == R]
    Xh = X.cpu().numpy()[order]
    Th = T.cpu().numpy()[order].astype(np.float64)
    groups = np.stack([Th[f:f + R] for f in full])  # (G, R, 3)
    return Xh[full], groups.mean(axis=1), groups


def _rel(pred, target):
    return float(np.linalg.norm(pred - target) / np.linalg.norm(target))


def test_trained_surrogate_beats_no_model_and_the_linear_closure():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_13267_amd import surrogate, train

    print(f"generating fresh samples: 32 starts x {R} replicas x 72 macro steps", flush=True)
    X, T, box_id, step_id, info = train.generate(32 * R, 72, equil=300, seed_k=97, replicas=R,
                                                 log=lambda *a, **k: None)
    Xg, Tm, groups = _replica_means(X, T, box_id, step_id)
    assert Xg.shape[0] > 500
    print("generating a separate fit set for the linear closure: 128 boxes x 72 macro steps", flush=True)
    Xf, Tf, _, _, _ = train.generate(128, 72, equil=300, seed_k=98, log=lambda *a, **k: None)
    members, nh, gscale, sscale = surrogate.load_trained()
    assert abs(gscale - train.GRAD_SCALE) < 1e-6 and abs(sscale - train.STRESS_SCALE) < 1e-9
    sur = surrogate.Surrogate(members, X.shape[1], nh, 3, max_batch=4096)
    Xd = torch.from_numpy(Xg).cuda()
    pred, _ = train.evaluate(sur, Xd, torch.from_numpy(Tm.astype(np.float32)).cuda(), 4096)
    pred = pred.cpu().numpy().astype(np.float64)
    sur.set_weights(surrogate.init_members(len(members), X.shape[1], nh, 3, seed=5))
    pred_u, _ = train.evaluate(sur, Xd, torch.from_numpy(Tm.astype(np.float32)).cuda(), 4096)
    pred_u = pred_u.cpu().numpy().astype(np.float64)
    sur.close()
    # linear closure of the newest gradient sample (4 components) with intercept
    hist = train.HIST
    cur_f = Xf[:, 4 * (hist - 1):4 * hist].double().cpu().numpy()
    A = np.concatenate([cur_f, np.ones((cur_f.shape[0], 1))], axis=1)
    coef, *_ = np.linalg.lstsq(A, Tf.double().cpu().numpy(), rcond=None)
    cur = Xg[:, 4 * (hist - 1):4 * hist].astype(np.float64)
    pred_lin = np.concatenate([cur, np.ones((cur.shape[0], 1))], axis=1) @ coef
    noise = float(np.sqrt(((groups - Tm[:, None]) ** 2).sum() / (R - 1) / R) / np.linalg.norm(Tm))
    e_tr, e_un, e_lin = _rel(pred, Tm), _rel(pred_u, Tm), _rel(pred_lin, Tm)
    print(f"against {R}-replica means ({Xg.shape[0]} rows): trained {e_tr:.4f}, linear closure {e_lin:.4f}, "
          f"untrained {e_un:.4f}, zero 1.0, noise left in the mean {noise:.4f}", flush=True)
    assert e_tr < 0.5 and e_tr < 0.5 * e_un
    assert e_tr < e_lin
    assert e_tr < 1.3 * noise
