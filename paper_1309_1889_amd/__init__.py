"""msmx: multilevel summation (MSM) electrostatics and parareal velocity
Verlet on an AMD Instinct MI355X.

Python binding of ``libmsmx.so`` (include/msm.h). The binding only marshals
arguments: every step of an evaluation runs in the library's HIP kernels.
PyTorch supplies device memory and the stream. Importing the package does not
load the library; the first call does, and fails loudly if it has not been
built (``python -m paper_1309_1889_amd.build``).
"""
from .binding import (  # noqa: F401
    MSM_FP32,
    MSM_FP64,
    MsmError,
    MsmContext,
    energy_forces_noalloc,
    lib,
    lib_path,
    parareal,
    parareal_window,
    status_string,
    WindowState,
)
from .autograd import msm_energy  # noqa: F401
