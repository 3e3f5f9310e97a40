"""Host logic of the learned proposal's run-level judge (no GPU): the fixed-step sampler's
reference ESS / J and held-out log predictive against a learned run's, window by window."""
import pytest

torch = pytest.importorskip("torch")


class FakeSampler:
    """Stands in for SMCSampler: J particles, a proposal switch and a scripted held-out score."""

    def __init__(self, J, heldout):
        self.J = J
        self.proposal = "learned"
        self.heldout = heldout  # {iteration: mean log predictive}
        self.k = 0
        self.switches = []

    def set_proposal(self, p):
        self.switches.append((self.k, p))
        self.proposal = p

    def predict(self, X, y):
        return {"accuracy": 1.0, "mean_log_pred": self.heldout[self.k]}


def _reference(PL, ess_frac, heldout, checkpoints=(5, 10, 15), runs=2):
    ref = PL.JudgeReference(None, None, checkpoints)
    for r in range(runs):
        ref.start_run()
        s = FakeSampler(100, heldout)
        s.proposal = "fixed"
        for k in range(1, len(ess_frac) + 1):
            s.k = k
            ref.record(s, k, 100 * ess_frac[k - 1])
    return ref


def _run(PL, ref, ess_frac, heldout):
    judge = PL.ProposalJudge(ref, ratio=0.9)
    s = FakeSampler(100, heldout)
    for k in range(1, len(ess_frac) + 1):
        s.k = k
        judge.after_step(s, k, 100 * ess_frac[k - 1])
    return judge, s


def test_judge_keeps_a_learned_move_that_matches_the_reference():
    from paper_2601_21983_amd import learned as PL
    held = {k: -0.1 for k in range(1, 11)}
    ref = _reference(PL, [0.4] * 10, held)
    judge, s = _run(PL, ref, [0.4] * 10, {k: -0.05 for k in range(1, 11)})
    rep = judge.report()
    assert not rep["fired"] and rep["learned_iterations"] == 10 and s.proposal == "learned"
    assert [c["iteration"] for c in rep["checks"]] == [5, 10]
    assert rep["checks"][0]["ess_frac_needed"] == pytest.approx(0.36)


def test_judge_falls_back_when_the_window_ess_drops():
    from paper_2601_21983_amd import learned as PL
    held = {k: -0.1 for k in range(1, 16)}
    ref = _reference(PL, [0.4] * 15, held)
    # iterations 6..10 at half the reference's ESS: the second window fails
    ess = [0.4] * 5 + [0.2] * 5 + [0.4] * 5
    judge, s = _run(PL, ref, ess, {k: 0.0 for k in range(1, 16)})
    rep = judge.report()
    assert rep["fired"] and rep["iteration"] == 10 and rep["reason"] == "ess"
    assert s.switches == [(10, "fixed")] and s.proposal == "fixed"
    # after the switch the run is a fixed-step run: no more learned iterations or checks
    assert rep["learned_iterations"] == 10 and len(rep["checks"]) == 2


def test_judge_falls_back_on_a_worse_heldout_score():
    from paper_2601_21983_amd import learned as PL
    ref = _reference(PL, [0.4] * 10, {k: -0.1 for k in range(1, 11)})
    judge, s = _run(PL, ref, [0.5] * 10, {k: -0.2 for k in range(1, 11)})
    rep = judge.report()
    assert rep["fired"] and rep["iteration"] == 5 and rep["reason"] == "heldout"


def test_judge_averages_over_the_window():
    from paper_2601_21983_amd import learned as PL
    ref = _reference(PL, [0.4] * 5, {k: -0.1 for k in range(1, 6)})
    # one poor iteration inside a window whose mean still reaches 0.9 x the reference
    judge, s = _run(PL, ref, [0.4, 0.4, 0.3, 0.4, 0.4], {k: -0.1 for k in range(1, 6)})
    assert not judge.report()["fired"]
    judge, s = _run(PL, ref, [0.4, 0.4, 0.0, 0.4, 0.4], {k: -0.1 for k in range(1, 6)})
    rep = judge.report()
    assert rep["fired"] and rep["reason"] == "ess"


def test_reference_averages_runs():
    from paper_2601_21983_amd import learned as PL
    ref = PL.JudgeReference(None, None, [2])
    for frac, held in [(0.2, -0.3), (0.4, -0.1)]:
        ref.start_run()
        s = FakeSampler(100, {1: held, 2: held})
        for k in (1, 2):
            s.k = k
            ref.record(s, k, 100 * frac)
    assert ref.runs == 2
    assert ref.ess_frac(1) == pytest.approx(0.3) and ref.heldout(2) == pytest.approx(-0.2)
    assert ref.covers(2) and not ref.covers(3)


def test_checkpoints_are_geometric():
    from paper_2601_21983_amd import learned as PL
    assert PL.judge_checkpoints(60) == [1, 2, 4, 8, 16, 32, 60]
    assert PL.judge_checkpoints(1) == [1]
    assert PL.judge_checkpoints(8) == [1, 2, 4, 8]


def test_judge_catches_a_losing_move_after_one_iteration():
    from paper_2601_21983_amd import learned as PL
    ref = _reference(PL, [0.4] * 8, {k: -0.1 for k in range(1, 9)}, checkpoints=PL.judge_checkpoints(8))
    judge, s = _run(PL, ref, [0.1] * 8, {k: -0.1 for k in range(1, 9)})
    rep = judge.report()
    assert rep["fired"] and rep["iteration"] == 1 and rep["learned_iterations"] == 1
    # windows between checkpoints: a move that matches keeps running through 1, 2, 4, 8
    judge, s = _run(PL, ref, [0.4] * 8, {k: -0.1 for k in range(1, 9)})
    assert [c["iteration"] for c in judge.report()["checks"]] == [1, 2, 4, 8]
