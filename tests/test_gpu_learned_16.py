"""The learned part at the throughput workload's size: 16^3 elements,
Re 1600, the P = 8 reference from t = 0, training pairs from t = 4 with
C4's training budget (50 snapshots, Adam batch 4096, 30 epochs), the
paper's network form (Algorithm 1's discrete-increment pairs, the three
momenta in and out, relu, correction after each step; Sec. 2.1, 2.2).

Over a window of 0.15 time units (the paper's windows are 0.15 - 0.3,
Table 1) the corrected P = 3 run stays closer to the filtered P = 8
solution (Eq. (9)) than the uncorrected one: measured 3.67e-2 against
7.07e-2.  Over C4's own window [4, 5] every network tried is worse than
the uncorrected run; the measured reason is recorded with the loss curves
in the design notes (the element-local network cannot follow the forcing
over a whole time unit at this Reynolds number)."""
import numpy as np
import pytest

from helpers import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_paper_form_gains_at_16cubed_re1600():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_11571_amd import study as st
    say("learned forcing 16^3 Re 1600, window 0.15, C4 training budget")
    res = st.run_study(N=16, Re=1600.0, t0=4.0, window=0.15, snapshots=50, eval_end=4.45, epochs=30, batch=4096,
                       orders=(), variants=[st.variant("alg1", "alg1", "momentum", "relu", "post", epochs=30)],
                       log=lambda *a: print("[study]", *a, flush=True))
    base, corr = res["runs"]["P3"], res["runs"]["P3+alg1"]
    losses = res["training"]["variants"]["alg1"]["loss_per_epoch"]
    print("P3 window error", base["mean_e_window"], "corrected", corr["mean_e_window"],
          "loss", losses[0], "->", losses[-1])
    assert losses[-1] < 0.1 * losses[0]
    assert corr["mean_e_window"] < 0.75 * base["mean_e_window"]
    # the correction costs one network evaluation per step
    assert corr["wall_per_unit_time_s"] < 2.0 * base["wall_per_unit_time_s"]
