"""Host logic of the burn-in driver (no GPU): the adaptation window schedules, and the
per-sampler settings every gradient sampler needs."""
import pytest

from paper_2606_04895_amd import driver


def test_doubling_schedule_of_1000_steps():
    assert driver.window_plan(1000) == [(10, True), (20, True), (40, True), (80, True),
                                        (160, True), (490, True), (200, False)]


@pytest.mark.parametrize("warmup", [1, 7, 39, 40, 41, 100, 333, 1000, 4096, 6000])
@pytest.mark.parametrize("schedule", ["doubling", "thirds"])
def test_windows_cover_the_warmup_exactly(warmup, schedule):
    plan = driver.window_plan(warmup, schedule)
    assert sum(w for w, _ in plan) == warmup
    assert all(w > 0 for w, _ in plan)
    assert plan[0][1]  # the first window always re-estimates the covariance
    if schedule == "thirds":
        assert all(upd for _, upd in plan) and len(plan) <= 3
    else:
        assert sum(1 for _, upd in plan if not upd) <= 1 and all(upd for _, upd in plan[:-1])


def test_every_gradient_sampler_has_its_settings():
    for s in ("mala", "hmc", "nuts"):
        assert 0 < driver.TARGET_ACCEPT[s] < 1 and driver.EPS0[s] > 0
        assert driver.SCHEDULE[s] in ("doubling", "thirds")
    assert driver.SCHEDULE["nuts"] == "doubling"
    assert 0 < driver.EPS_FLOOR < 1e-6
    assert driver.window_plan(0) == []
