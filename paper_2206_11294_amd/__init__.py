"""MI355X-native multigrid solver for the coupled pressure-temperature
system of an all-Mach VoF time step (HIP library libptmg + thin binding)."""
from .ptmg import (PT_COEF_EXPLICIT, PT_COEF_PHASES, PT_PREC_FP64, PT_PREC_MIXED,  # noqa: F401
                   PtMg, PtMgError, copy_kernel, footprint_bytes, lib, phase_struct,
                   pt_phase, pt_problem)
