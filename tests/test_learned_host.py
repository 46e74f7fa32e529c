"""Host logic of the learned-proposal driver (no GPU): the audit's verdict."""
import torch

from paper_1409_4256_amd import learned


class _Plan:
    def __init__(self, n_audit):
        self.n_audit = n_audit


def _iteration(n_audit, recall):
    it = learned.ProposedIteration.__new__(learned.ProposedIteration)
    it.plan = _Plan(n_audit)
    it.recall = torch.tensor([recall], dtype=torch.float64)
    return it


def test_accepted_needs_a_finite_recall_when_frames_are_audited():
    """No audited frames: no verdict (accepted).  With audited frames, a recall below
    0.98 or not a finite number (a broken iteration) rejects."""
    for n_audit, rec, want in ((0, float("nan"), True), (5, float("nan"), False), (5, 0.99, True),
                               (5, 0.98, True), (5, 0.5, False), (5, float("inf"), False)):
        assert _iteration(n_audit, rec).accepted() == want, (n_audit, rec)


def test_proposed_or_full_runs_the_full_search_only_on_rejection():
    calls = []

    class _Prop:
        def __init__(self, n_audit, recall):
            self.it = _iteration(n_audit, recall)

        def step(self, a, b, ev=None):
            calls.append("proposed")

        def accepted(self):
            return self.it.accepted()

    full = lambda a, b: calls.append("full")
    assert learned.proposed_or_full(_Prop(4, 0.999), full, None, None) is True
    assert calls == ["proposed"]
    calls.clear()
    assert learned.proposed_or_full(_Prop(4, 0.9), full, None, None) is False
    assert calls == ["proposed", "full"]
