"""The live loop's overrun count, driven on the CPU by a fake frame clock."""
import pytest

from paper_2509_25924_amd.live import LiveLoop, max_overrun_free_rate


class FakeClock:
    """Time moves only when the loop waits for a frame or the processing reports its duration."""

    def __init__(self):
        self.t = 100.0

    def now(self):
        return self.t

    def sleep_until(self, t):
        self.t = max(self.t, t)


def _loop(service, period, buffer_frames=1):
    clk = FakeClock()

    def process(k):
        clk.t += service(k)
    return LiveLoop(process, period, clock=clk, buffer_frames=buffer_frames)


def test_no_overrun_when_processing_is_faster_than_the_camera():
    st = _loop(lambda k: 0.009, 0.01).run(100)
    assert st.frames == 100 and st.overruns == 0
    assert st.max_lateness_s == pytest.approx(-0.001)
    assert all(c == pytest.approx(0.009) for c in st.completion_s)


def test_every_frame_overruns_when_processing_is_slower():
    st = _loop(lambda k: 0.012, 0.01).run(50)
    assert st.overruns == 50               # even frame 0 is not done when frame 1 arrives
    assert st.completion_s[-1] > st.completion_s[1]   # the backlog grows


def test_one_slow_frame_and_recovery():
    # 20 ms once in a 10 ms cadence, 5 ms otherwise: frame 3 finishes 10 ms after its deadline, frame 4
    # starts 10 ms late and finishes 5 ms late, frame 5 is on time again
    st = _loop(lambda k: 0.020 if k == 3 else 0.005, 0.01).run(10)
    assert st.overruns == 2
    assert st.max_lateness_s == pytest.approx(0.010)
    st2 = _loop(lambda k: 0.020 if k == 3 else 0.005, 0.01, buffer_frames=2).run(10)
    assert st2.overruns == 0               # a two-frame buffer absorbs it


def test_exactly_on_the_deadline_is_not_an_overrun():
    st = _loop(lambda k: 1 / 64, 1 / 64).run(20)     # binary-exact times: no rounding at the tie
    assert st.overruns == 0 and st.max_lateness_s == 0.0


def test_max_overrun_free_rate_sweep():
    res = max_overrun_free_rate(lambda p: _loop(lambda k: 1 / 256, p), [64, 128, 256, 512, 1024], 40)
    assert res["max_overrun_free_hz"] == 256
    assert [r["overruns"] > 0 for r in res["rates"]] == [False, False, False, True, True]


def test_arguments_are_checked():
    with pytest.raises(ValueError):
        LiveLoop(lambda k: None, 0.0)
    with pytest.raises(ValueError):
        LiveLoop(lambda k: None, 0.01, buffer_frames=0)
