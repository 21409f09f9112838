"""The learned surrogate end to end at reduced size: dataset from the
simulator, training on the library's MFMA kernels, screening with the
simulator as judge.  What the network gains over the method without it:
ranking held-out robots by prediction finds far more of the truly best
robots than the same simulation budget spent on random robots."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_surrogate_screening_beats_random_at_equal_budget():
    from paper_1911_10274_amd import scenes
    from paper_1911_10274_amd import surrogate as S

    Xt, Yt, _ = S.dataset(16384, seed=5)
    eval_batch = scenes.small_robot_batch(2000, S.chunk_seed(50, 0))
    Ye, _ = S.simulate(eval_batch)
    Xe = S.featurize(eval_batch)
    model = S.Surrogate(seed=3)
    fit = model.fit(Xt, Yt, epochs=12, batch=512, lr=1e-3, X_val=Xe, Y_val=Ye)
    hist, val = fit["train_loss"], fit["val_loss"]
    assert hist[-1] < hist[0] and len(val) == 12
    # it learns something that carries over to robots it has not seen: the
    # held-out loss (standardised MSE, 1 for predicting the mean) falls below 1
    assert val[-1] < 0.95 * val[0] and val[-1] < 1.0
    res = S.screen(model, Xe, Ye, eval_batch, frac=0.05)
    model.close()
    print(res)
    # the judge (re-simulation of the picked robots on their own, plain
    # engine) reproduces the dataset's values for them exactly
    assert res["judge_matches_dataset"]
    assert res["spearman_dx"] > 0.15
    assert res["recall_top"] >= 2 * res["recall_random_expected"]
    assert res["mean_picked_dx"] > res["mean_random_dx"]
