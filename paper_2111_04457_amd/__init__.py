"""MI355X (gfx950) library for the Wilson / Wilson-clover fermion matrix of
eq. (1) of the Bridge++ 2.0 paper (arXiv:2111.04457) and its Krylov solvers.

The compute path is the HIP library liblq.so behind the C ABI of
include/lq.h; this package only marshals torch tensors and streams to it.
"""
from ._lib import LQError, load  # noqa: F401

__all__ = ["Operator", "Field", "Batch", "SolverParams", "SolveStats", "apply_field", "pf_force", "PseudofermionAction",
           "MDParams", "MDStats", "gauge_force", "md_trajectory", "hmc_step", "workspace_bytes", "bandwidth_probe",
           "Multigrid", "MGParams", "LQError", "load"]


def __getattr__(name):
    if name in ("Operator", "Field", "Batch", "SolverParams", "SolveStats", "apply_field", "pf_force",
                "PseudofermionAction", "MDParams", "MDStats", "gauge_force", "md_trajectory", "hmc_step",
                "workspace_bytes", "bandwidth_probe", "Multigrid", "MGParams"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
