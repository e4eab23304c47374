"""Seeded synthetic inputs (fields, shifts, schedules, right-hand sides,
request traces).  Holds no solver arithmetic; used by the oracle, the tests,
the benchmark and the GPU library alike."""
from .inputs import *  # noqa: F401,F403
