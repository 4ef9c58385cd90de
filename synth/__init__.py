"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This package evaluates the paper's received-signal model (Sec. II) for given
target trajectories and draws noise.  It holds none of the search method's
arithmetic (no lattice, offsets, de-ramp or fine phases).
"""
from .echo import (RadarParams, Target, CONFIGS, PD_SCENARIO, config_case,  # noqa: F401
                   draw_targets, make_echo, impulse_target_echo,
                   adjoint_candidates)
