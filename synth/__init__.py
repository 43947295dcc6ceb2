"""Seeded synthetic inputs for the state-vector path.

This package only *draws* inputs: gate lists, initial states and arithmetic
parameters. It applies no gate, performs no transform and reduces nothing, so
the CPU oracle and the GPU library can both consume its output without
sharing any of the simulation arithmetic.
"""
from .circuits import *  # noqa: F401,F403
