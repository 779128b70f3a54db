"""What the trained proposal network gains over the method without it: a
network trained on the GPU by the library's own kernels, on trials labelled by
the plain full-grid search, then the learned path against the plain FP32 grid
search on the same held-out trials. The gain is counted in grid points
evaluated (timing is reported, not asserted), at equal accuracy: equal RMSE,
and in the paired comparison on the same trials equal median error, resolved
fraction and RMSE over resolved sources."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2604_19723_amd import bartlett as bb
from paper_2604_19723_amd import learned as lr
from paper_2604_19723_amd import workload as wl

pytestmark = pytest.mark.gpu
DEV = "cuda"


def test_trained_network_cuts_the_grid_at_equal_rmse():
    grid = wl.ula_grid(lr.G)
    plan = bb.ba_plan_create(lr.M, wl.ula_positions(lr.M), bb.BA_GRID_ULA_DEG, lr.G, grid, lr.G, 1, 0)
    net = bb.ba_mlp_create(lr.M * lr.M, 512, 3, lr.K, 16384, bb.BA_PREC_BF16, 21)
    try:
        X, U, Mk = lr.make_training_set(plan, 262144, 0xBA57_00F1, DEV)
        hist = lr.train(net, X, U, Mk, epochs=6, batch=1024, lr=1e-3, seed=3)
        del X, U, Mk
        torch.cuda.empty_cache()
        assert hist[-1] < hist[0], hist
        # the threshold is chosen on a validation set, then judged on held-out trials
        taus = [0.0, 0.02, 0.05, 0.1, 0.15, 0.2, 0.25, 0.3]
        val = lr.evaluate(plan, net, wl.config5(1400, seed_offset=6, snr_db=wl.C2_SNRS), taus, DEV)
        best = lr.choose_tau(val)
        assert best is not None, [(r["tau"], r["rmse"], r["fallback"], r["accuracy_vs_plain"]["equal"])
                                  for r in val["learned"]]
        tau = best["tau"]
        ev = lr.evaluate(plan, net, wl.config5(1400, seed_offset=7, snr_db=wl.C2_SNRS), [tau], DEV)
        plain, learned = ev["plain"], ev["learned"][0]
        # the window kernel projects every 16-column block a window touches:
        # at most (2 hw) / 16 + 2 blocks per window, i.e. 128 points for hw = 50
        hw = 50
        pts = lr.K * 16 * ((2 * hw) // 16 + 2)
        frac = (1 - learned["fallback"]) * pts / lr.G + learned["fallback"]
        frac_window = (1 - learned["fallback"]) * (lr.K * (2 * hw + 1)) / lr.G + learned["fallback"]
        print("tau %.2f; plain RMSE %.4f (SE %.4f) %.0f trials/s; learned RMSE %.4f (SE %.4f) %.0f trials/s, "
              "fallback %.3f, grid evaluated %.3f (block-rounded; %.3f in window points)" % (
                  tau, plain["rmse"]["rmse"], plain["rmse"]["se"], plain["trials_per_s"], learned["rmse"]["rmse"],
                  learned["rmse"]["se"], learned["trials_per_s"], learned["fallback"], frac, frac_window))
        acc = learned["accuracy_vs_plain"]
        print("paired accuracy vs plain: diff %s, paired SE %s, index identity %.4f" % (
            acc["diff"], acc["diff_se"], learned["index_identity_vs_plain"]))
        assert lr.equal_accuracy(learned, plain), acc["equal"]
        assert frac < 0.5
    finally:
        net.close()
        plan.close()
