"""The deferred-update trigger (Sec. 5.2.2) driven by forced throughput series (no GPU)."""
import pytest

from paper_2601_03187_amd.deferred import DeferredUpdate


def test_first_window_is_the_baseline_and_drops_within_tau_do_nothing():
    p = DeferredUpdate(tau=0.05, theta=100)
    assert [p.observe(x, 0) for x in (100.0, 99.0, 96.0, 95.01)] == [None] * 4
    assert p.th_base == 100.0


def test_drop_beyond_tau_picks_incremental_or_full_by_theta():
    p = DeferredUpdate(tau=0.05, theta=100)
    p.observe(100.0, 0)
    assert p.observe(94.0, 100) == "incremental"  # 6% drop, theta not exceeded
    assert p.observe(94.0, 101) == "full"         # same drop, more coarse rules than theta


def test_incremental_keeps_the_baseline_full_resets_it():
    p = DeferredUpdate(tau=0.05, theta=10)
    p.observe(200.0, 0)
    assert p.observe(180.0, 0) == "incremental"
    p.deployed("incremental")
    assert p.observe(195.0, 0) is None            # measured against the old base (200)
    assert p.observe(189.0, 50) == "full"
    p.deployed("full")
    assert p.observe(120.0, 0) is None            # the first window after: new baseline
    assert p.th_base == 120.0
    assert p.observe(113.0, 0) == "incremental"   # 5.8% below the new base


def test_bad_arguments():
    with pytest.raises(ValueError):
        DeferredUpdate(tau=0.0)
    with pytest.raises(ValueError):
        DeferredUpdate().deployed("sometimes")
