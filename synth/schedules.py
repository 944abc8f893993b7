"""Temperature and field schedules of the benchmark workloads (k_B = 1, as in
the paper's "File Formats" section)."""
import numpy as np


def cooling_schedule(n_steps=20, T_hi=3.0, T_lo=0.1):
    """n_steps temperatures linearly from T_hi down to T_lo."""
    return T_hi + (T_lo - T_hi) * np.arange(n_steps) / max(n_steps - 1, 1)


def replica_temperatures(n_rep=64, T_lo=0.1, T_hi=3.0):
    """One temperature per replica, linearly from T_lo up to T_hi."""
    return T_lo + (T_hi - T_lo) * np.arange(n_rep) / max(n_rep - 1, 1)


def hysteresis_fields(n_steps=401, B_max=2.0):
    """Field swept +B_max -> -B_max -> +B_max in n_steps (odd) steps."""
    half = (n_steps - 1) // 2
    down = B_max - 2 * B_max * np.arange(half + 1) / half
    up = -B_max + 2 * B_max * np.arange(1, half + 1) / half
    return np.concatenate([down, up])
