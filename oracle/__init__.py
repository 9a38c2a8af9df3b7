"""FP64 CPU oracle for the multilevel summation method and the parareal
integrator built on it.

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg are the only callers. Nothing here is imported by
the product package, and this package imports nothing from it.

``libmsm_oracle.so`` is plain C (see ``msm_oracle.c``); this module is the
ctypes loader plus NumPy conveniences. ``dense.py`` holds an independent dense
matrix evaluation of the paper's nested interpolation formula, used to pin the
fast oracle on tiny inputs.
"""
from .loader import (  # noqa: F401
    OracleParams,
    METHOD_MSM,
    METHOD_CUTOFF,
    METHOD_WOLF,
    lib,
    gamma,
    dgamma,
    Phi,
    dPhi,
    gstar,
    glevel,
    levels,
    grid_shape,
    msm,
    coulomb,
    cutoff,
    cutoff_subset,
    wolf,
    short_subset,
    threads,
    set_threads,
    OracleModel,
    md_forces,
    md_forces_split,
    vv_mts,
    vv,
    parareal,
    parareal_window,
    window_buffers,
    WindowState,
)
