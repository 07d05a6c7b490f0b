"""BC-FMM Galerkin volume potentials on MI355X: Python binding of libbcvol (see include/bcv.h)."""

from .bcv import (  # noqa: F401
    BCVError,
    FP64,
    MIXED_F32,
    NEAR_ASSEMBLED,
    NEAR_QUADRATURE,
    PART_FAR,
    PART_NEAR,
    TOUCH_CLASSES,
    build_bc_tree,
    btv_apply,
    lib,
    PHASES,
    plan_enable_timing,
    plan_interactions,
    plan_phase_times,
    touching_integrals,
    vtb_apply,
    vtv_apply,
    vtv_apply_parts,
)
