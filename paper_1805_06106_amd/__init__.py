"""MI355X (gfx950) GIGAQBX: FMM-accelerated QBX for 3D Laplace layer potentials.

The compute path is the HIP library libgigaqbx.so (C ABI in include/gigaqbx.h); this
package only binds it.  There is no CPU fallback: using a plan without the built library
raises.
"""

from ._capi import (  # noqa: F401
    GQ_FLAG_HOST_ONLY,
    GQ_FLAG_TIMING,
    GQ_TARGET_FAR,
    GQ_TARGET_UNMATCHED,
    GQError,
    gq_associate_targets as associate_targets,
    gq_points_near as points_near,
    gq_apply,
    gq_last_error,
    gq_list_export,
    gq_plan_create,
    gq_plan_destroy,
    gq_qbx_locals,
    gq_stats,
    gq_translation_matrix,
    gq_tree_export,
    make_params,
)
from .plan import Plan  # noqa: F401
