"""MI355X trapped-ion engine: all-pairs Coulomb field + linear Paul trap field +
damped velocity-Verlet steps in HIP kernels behind the C ABI of include/lion.h."""
from .lion import (LION_FP64, LION_MIXED_F64ACC, LION_MIXED_KAHAN, PRECISIONS, LionError,
                   Simulation, load)

__all__ = ["LION_FP64", "LION_MIXED_F64ACC", "LION_MIXED_KAHAN", "PRECISIONS", "LionError",
           "Simulation", "load"]
