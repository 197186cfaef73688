"""Deferred update policy (Sec. 5.2.2), host side.

Immediate updates (Sec. 5.2.1, ``tang_insert`` / ``tang_delete``) keep the tuple set, so
the predictor stays valid but drifts from the rules: inserted rules sit in coarser tuples
and traffic to them is predicted less well, which shows up as lower throughput (more
fallback probes). The policy watches the classification throughput of each window:
``th_base`` is the first window after the last full retraining, and when
1 - th_cur / th_base exceeds tau an update is due. It is a full retraining (rebuild the
tuple space from the live rules, train from scratch) when more than theta live rules sit
in a tuple coarser than their own signature (``tang_ruleset_coarse_rules``), otherwise
an incremental training (fine-tune the current model on fresh labels from the current
tuple space). A full retraining starts a new baseline; an incremental one keeps it.
"""
from __future__ import annotations


class DeferredUpdate:
    def __init__(self, tau: float = 0.05, theta: int = 10_000):
        if not 0.0 < tau < 1.0:
            raise ValueError("tau must be in (0, 1)")
        self.tau = tau
        self.theta = theta
        self.th_base: float | None = None

    def observe(self, th_cur: float, coarse_rules: int) -> str | None:
        """Throughput of one window (any unit); returns None, "incremental" or "full"."""
        if self.th_base is None:
            self.th_base = th_cur
            return None
        if 1.0 - th_cur / self.th_base > self.tau:
            return "full" if coarse_rules > self.theta else "incremental"
        return None

    def deployed(self, action: str) -> None:
        """Called once the update an ``observe`` asked for is in place."""
        if action == "full":
            self.th_base = None
        elif action != "incremental":
            raise ValueError(action)
