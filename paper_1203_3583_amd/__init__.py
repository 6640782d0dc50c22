"""MI355X (gfx950) arbitrary-shape-surface Fresnel diffraction.

The forward transform of Shimobaba, Masuda and Ito, "Arbitrary shape surface
Fresnel diffraction" (Sec. 2, Eq. (7)-(9)) as a 2D type-1 non-uniform FFT in
hand-written HIP kernels behind the C ABI of include/asf.h, and its adjoint (the
type-2 direction) for gradients.  ``asf.Plan`` is the Python handle;
``asf.LinePlan`` the one-dimensional (profile) form;
``autograd.propagate`` is the differentiable forward; ``csrc/build.py`` builds
``libasf.so``.
"""
from .asf import (AsfError, LinePlan, Plan, STAGES, lib, last_error, make_line_params,  # noqa: F401
                  make_params, workspace_bytes)
from .autograd import energy_matched, intensity_loss, phase_descent, propagate  # noqa: F401

__all__ = ["AsfError", "Plan", "LinePlan", "make_line_params", "STAGES", "lib", "last_error", "make_params", "workspace_bytes",
           "propagate", "intensity_loss", "energy_matched", "phase_descent"]
