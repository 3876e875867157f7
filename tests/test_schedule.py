"""Host checks of the schedules (no GPU): the H-LU of a small grid is
recorded and scheduled by the library, then checked against the run rules
alone (hm_schedule_check): every pair of operations that touch overlapping
rows of one object, one of them writing, must be ordered by stream order,
event waits or epoch joins (dataflow), or by wave order (waves); every pair
of temporaries that share memory must be ordered as wholes; every event
waited for must be recorded; every item must sit in exactly one launch."""
import pytest

from paper_1703_09085_amd import hm

CASES = [(2, 32, 8), (3, 12, 16)]


@pytest.mark.parametrize("dim,side,leaf", CASES)
@pytest.mark.parametrize("mode", ["standard", "accumulated", "fused"])
@pytest.mark.parametrize("schedule,epoch_ms", [("waves", None), ("dataflow", "25"), ("dataflow", "0.2")])
def test_schedule_orders_every_conflict(monkeypatch, dim, side, leaf, mode, schedule, epoch_ms):
    monkeypatch.delenv("HM_SCHEDULE", raising=False)
    if epoch_ms is not None:
        monkeypatch.setenv("HM_DF_EPOCH_MS", epoch_ms)
    r = hm.schedule_check(dim, side, leaf, mode=mode, schedule=schedule)
    print(dim, side, leaf, mode, schedule, epoch_ms, r)
    assert r["dataflow"] == (schedule == "dataflow")
    assert r["conflicts"] > 0 and r["launches"] > 0
    assert r["unordered"] == 0
    assert r["unordered_temporaries"] == 0
    assert r["missing_events"] == 0
    assert r["misplaced_items"] == 0
    if epoch_ms == "0.2":
        assert r["shared_temporaries"] > 0  # short epochs: memory is reused across epochs


def test_schedule_check_rejects_bad_arguments():
    with pytest.raises(hm.HMError):
        hm.schedule_check(4, 8, 4)
    with pytest.raises(hm.HMError):
        hm.schedule_check(2, 8, 0)
    with pytest.raises(KeyError):
        hm.schedule_check(2, 8, 4, schedule="sideways")
