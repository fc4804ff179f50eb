"""Live acquisition loop with the paper's overrun criterion (host logic).

The paper's live measurements (section "Live (Real-Time) computing
performances") feed camera frames to the estimator at a fixed rate and raise
the rate until overruns appear: frames the processing could not keep up
with.  This module models that loop: frame k arrives at t0 + k * period;
its pair is processed once it has arrived and the previous frame's
processing has finished; the frame overruns when its processing completes
after its deadline, its arrival plus `buffer_frames` periods (the frames the
acquisition can hold before it must drop one).

The clock is injectable: `MonotonicClock` is the real one, and tests drive
the loop with a fake clock whose time only moves when the loop waits or the
processing reports its duration, so the overrun count of any schedule can be
checked on the CPU.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional


class MonotonicClock:
    """Wall clock (time.perf_counter) with a sleep that waits until a given time."""

    def now(self) -> float:
        return time.perf_counter()

    def sleep_until(self, t: float) -> None:
        while True:
            d = t - time.perf_counter()
            if d <= 0:
                return
            time.sleep(d if d > 2e-3 else 0)   # sleep coarse, spin the last 2 ms


@dataclass
class LiveStats:
    frames: int = 0
    overruns: int = 0
    max_lateness_s: float = 0.0       # completion minus deadline, worst frame (<= 0 when none overran)
    completion_s: List[float] = field(default_factory=list)   # per frame: completion minus arrival

    @property
    def overrun_free(self) -> bool:
        return self.overruns == 0


class LiveLoop:
    """Runs `process(k)` for frames k = 0 .. n-1 arriving every `period` seconds.

    process(k) enqueues the work of frame k; wait() blocks until it has
    completed (for the GPU path: a stream synchronisation).  A frame
    overruns when wait() returns after arrival + buffer_frames * period.
    """

    def __init__(self, process: Callable[[int], None], period: float, wait: Optional[Callable[[], None]] = None,
                 clock=None, buffer_frames: int = 1):
        if not period > 0:
            raise ValueError("period must be > 0")
        if buffer_frames < 1:
            raise ValueError("buffer_frames must be >= 1")
        self.process = process
        self.wait = wait or (lambda: None)
        self.period = float(period)
        self.clock = clock or MonotonicClock()
        self.buffer_frames = int(buffer_frames)

    def run(self, n_frames: int) -> LiveStats:
        st = LiveStats()
        t0 = self.clock.now()
        for k in range(n_frames):
            arrival = t0 + k * self.period
            self.clock.sleep_until(arrival)      # returns at once when processing is behind
            self.process(k)
            self.wait()
            done = self.clock.now()
            late = done - (arrival + self.buffer_frames * self.period)
            st.frames += 1
            st.completion_s.append(done - arrival)
            if late > 0:
                st.overruns += 1
            st.max_lateness_s = late if st.frames == 1 else max(st.max_lateness_s, late)
        return st


def max_overrun_free_rate(make_loop: Callable[[float], LiveLoop], rates: List[float], n_frames: int) -> dict:
    """The paper's procedure: run the loop at increasing frame rates (Hz) and report the overruns at each;
    the highest rate without any is the live rate."""
    rows, best = [], None
    for r in sorted(rates):
        st = make_loop(1.0 / r).run(n_frames)
        rows.append({"rate_hz": r, "overruns": st.overruns, "frames": st.frames,
                     "max_lateness_ms": round(st.max_lateness_s * 1e3, 3)})
        if st.overrun_free:
            best = r
    return {"rates": rows, "max_overrun_free_hz": best}
