"""Host-side logic of the serving loop: HBM-footprint admission (no GPU needed)."""
import pytest

from paper_1304_7211_amd.serve import AdmissionController


def test_admission_budget_and_slots():
    c = AdmissionController(budget_bytes=100, max_slots=3)
    assert c.try_admit(40) and c.try_admit(40)
    assert not c.try_admit(30)          # budget: 80 + 30 > 100
    assert c.try_admit(20)              # exactly 100
    assert not c.try_admit(0)           # slots exhausted
    c.release(40)
    assert c.try_admit(30)
    assert c.peak_used == 100 and c.peak_slots == 3


def test_admission_never_fits():
    c = AdmissionController(budget_bytes=1, max_slots=8)
    assert not c.fits_ever(2)
    assert c.fits_ever(1)
    assert not c.try_admit(2)
    assert c.used == 0 and c.slots == 0


def test_release_underflow_is_caught():
    c = AdmissionController(budget_bytes=10, max_slots=2)
    with pytest.raises(AssertionError):
        c.release(5)
