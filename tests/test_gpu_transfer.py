"""Transfer learning of the corrective forcing (Sec. 3.5) on the GPU: a
network trained on one time frame or Reynolds number, applied to another
directly, after a short retraining that starts from its weights, and
against a network trained on the target frame from scratch (Algorithm 1
pairs and correction, all five variables, tanh; 8^3 elements, P_HO = 8,
P_LO = 3, window 0.15 with one snapshot per low-order step, evaluation over
0.3 time units).

Parity unpinned: the paper's transfer figures are not available; what is
tested is the paper's qualitative finding with this project's own runs --
retraining from transferred weights for a quarter of the epochs reaches an
accuracy close to training from scratch (at least 90 % of its error
reduction over the uncorrected low order), for a quarter of the training
time.
"""
import pytest

from helpers import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = {"time frame (Re 200, t 4 -> 7)": ((200.0, 4.0), (200.0, 7.0)),
         "Reynolds number (1600 -> 200, t 4)": ((1600.0, 4.0), (200.0, 4.0))}


@pytest.fixture(scope="module", params=list(CASES))
def transfer(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_11571_amd import study as st
    say("transfer", request.param)
    source, target = CASES[request.param]
    return st.run_transfer(N=8, P_lo=3, source=source, target=target, window=0.15, snapshots=100, eval_span=0.3,
                           retrain_epochs=50, batch=512, log=lambda *a: print("[study]", *a, flush=True))


def test_retraining_reaches_scratch_accuracy_faster(transfer):
    runs = transfer["runs"]
    p3, src, ret, scr = runs["P3"], runs["P3+source"], runs["P3+retrained"], runs["P3+scratch"]
    print("mean e window: P3 %.3e source %.3e retrained %.3e scratch %.3e" % (
        p3["mean_e_window"], src["mean_e_window"], ret["mean_e_window"], scr["mean_e_window"]))
    print("training s: retrained %.2f scratch %.2f" % (transfer["training_seconds"]["retrained"],
                                                       transfer["training_seconds"]["scratch"]))
    assert ret["mean_e_window"] < 0.2 * p3["mean_e_window"]
    # "close to training from scratch": the retrained network recovers at
    # least 90 % of the error reduction that training from scratch achieves
    # over the uncorrected low order (measured 96 % and 95 %)
    gap = p3["mean_e_window"] - scr["mean_e_window"]
    assert ret["mean_e_window"] < scr["mean_e_window"] + 0.1 * gap
    assert ret["mean_e_beyond"] < 0.5 * p3["mean_e_beyond"]
    assert transfer["training_seconds"]["retrained"] < 0.4 * transfer["training_seconds"]["scratch"]


def test_online_retraining_loop():
    """The retraining loop of the paper's outlook: a P = 8 shadow run
    measures the error of the corrected P = 3 run at Re 200 from t = 4 to 7;
    whenever e_n exceeds the tolerance the network is retrained from its
    current weights on a fresh 0.075-long window and the low order is
    re-matched to the filtered P = 8 state.  Retraining must beat re-matching alone, the first network
    alone and the uncorrected low order, and keep e_n near the tolerance."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_11571_amd import study as st
    say("online retraining loop")
    tol = 3e-2
    res = st.run_online(N=8, Re=200.0, P_lo=3, t0=4.0, t_end=7.0, window=0.15, snapshots=100, tol=tol,
                        retrain_epochs=50, batch=512, log=lambda *a: print("[study]", *a, flush=True))
    m = res["mean_e"]
    print("mean e_n: online %.3e rematched %.3e fixed %.3e uncorrected %.3e; %d retrains, high order on %.0f %% "
          "of the span" % (m["online"], m["rematched"], m["fixed"], m["uncorrected"], len(res["retrains"]),
                           100 * res["high_order_fraction_of_span"]))
    assert len(res["retrains"]) >= 1
    assert m["online"] < 0.25 * m["rematched"]
    assert m["online"] < 0.1 * m["uncorrected"]
    assert res["max_e"]["online"] < 2 * tol
