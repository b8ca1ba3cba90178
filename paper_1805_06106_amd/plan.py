"""Convenience wrapper owning a plan handle (argument marshalling only)."""

from __future__ import annotations

from . import _capi as C


class Plan:
    """A GIGAQBX plan for fixed geometry; apply() evaluates densities on the GPU.

    Geometry arrays are numpy (N,3)/(N,) float64; densities/potentials are torch tensors on
    the GPU, shaped (n_densities, n_src) / (n_densities, n_tgt), float64.
    """

    def __init__(self, *, src_xyz, src_w, src_normal, ctr_xyz, ctr_radius, tgt_xyz, tgt_center,
                 p_qbx, p_fmm, kernel="S", nmax=512, tcf=0.9, n_densities=1, timing=False,
                 host_only=False, lists=None, wfar_direct_max=0, precision="fp64",
                 graph=False, autotune=False, tcr_norm="l2", level_restrict=False,
                 m2l_rotation=False, overlap=False, max_device_bytes=0, deterministic=False,
                 autotune_tree=False, stream=None):
        flags = ((C.GQ_FLAG_TIMING if timing else 0) | (C.GQ_FLAG_HOST_ONLY if host_only else 0)
                 | (C.GQ_FLAG_GRAPH if graph else 0) | (C.GQ_FLAG_AUTOTUNE if autotune else 0)
                 | (C.GQ_FLAG_DETERMINISTIC if deterministic else 0)
                 | (C.GQ_FLAG_AUTOTUNE_TREE if autotune_tree else 0))
        self.params = C.make_params(p_qbx, p_fmm, nmax=nmax, tcf=tcf, kernel=kernel,
                                    n_densities=n_densities, flags=flags, lists=lists,
                                    wfar_direct_max=wfar_direct_max, precision=precision,
                                    tcr_norm=tcr_norm, level_restrict=level_restrict,
                                    m2l_rotation=m2l_rotation,
                                    max_device_bytes=max_device_bytes)
        self.n_src = int(src_xyz.shape[0])
        self.n_ctr = int(ctr_xyz.shape[0])
        self.n_tgt = int(tgt_xyz.shape[0])
        self.p_qbx = int(p_qbx)
        self.n_densities = int(n_densities)
        self.n_density_cols = self.n_src  # node values per density row
        self.handle = None
        self.handle = C.gq_plan_create(self.params, src_xyz, src_w, src_normal, ctr_xyz,
                                       ctr_radius, tgt_xyz, tgt_center, stream=stream)
        if overlap:
            self.set_overlap(True)

    @classmethod
    def from_workload(cls, w, **kw):
        args = dict(p_qbx=w.p_qbx, p_fmm=w.p_fmm, kernel=w.kernel, nmax=w.nmax, tcf=w.tcf)
        args.update(kw)
        plan = cls(src_xyz=w.src_xyz, src_w=w.src_w, src_normal=w.src_normal, ctr_xyz=w.ctr_xyz,
                   ctr_radius=w.ctr_radius, tgt_xyz=w.tgt_xyz, tgt_center=w.tgt_center, **args)
        if getattr(w, "interp", None) is not None and not args.get("host_only", False):
            plan.set_source_interp(w.n_elem, w.interp)
        return plan

    @classmethod
    def batch(cls, plans, *, timing=False, graph=False, autotune=False, overlap=False,
              stream=None):
        """Merge plans (same orders, kernel, precision and density count) into one plan whose
        density/potential rows are the members' rows concatenated in the order given."""
        self = cls.__new__(cls)
        flags = ((C.GQ_FLAG_TIMING if timing else 0) | (C.GQ_FLAG_GRAPH if graph else 0)
                 | (C.GQ_FLAG_AUTOTUNE if autotune else 0))
        self.handle = None
        self.handle = C.gq_batch_create([p.handle for p in plans], flags, stream=stream)
        self.params = plans[0].params
        self.n_src = sum(p.n_src for p in plans)
        self.n_ctr = sum(p.n_ctr for p in plans)
        self.n_tgt = sum(p.n_tgt for p in plans)
        self.p_qbx = plans[0].p_qbx
        self.n_densities = plans[0].n_densities
        self.n_density_cols = self.n_src
        if overlap:
            self.set_overlap(True)
        return self

    def apply(self, density, potential=None, stream=None):
        import torch

        if potential is None:
            potential = torch.empty((self.n_densities, self.n_tgt), dtype=torch.float64,
                                    device=density.device)
        if density.dtype != torch.float64 or not density.is_contiguous():
            raise ValueError("density must be a contiguous float64 device tensor")
        want = (self.n_densities, self.n_density_cols)
        if tuple(density.shape) != want:
            raise ValueError(f"density shape {tuple(density.shape)} != {want}")
        C.gq_apply(self.handle, density, potential, stream=stream)
        return potential

    def set_overlap(self, on):
        """Run the far-field chain on a second stream beside the near field (True) or every
        stage in order on the apply stream (False, the default)."""
        C.gq_set_overlap(self.handle, 1 if on else 0)

    def set_target_normals(self, normals):
        """Target normals (n_tgt, 3) for the adjoint double layer (kernel "SP")."""
        C.gq_set_target_normals(self.handle, normals)

    def set_source_interp(self, n_elem, interp):
        """Oversampled quadrature: the sources are n_elem elements' quadrature nodes
        (element-major) and densities become node values, (n_densities, n_elem * n_node);
        interp (n_quad, n_node) maps one element's node values to its quadrature nodes."""
        C.gq_set_source_interp(self.handle, n_elem, interp)
        self.n_density_cols = int(n_elem) * int(interp.shape[1])

    def stats(self):
        return C.gq_stats(self.handle)

    def qbx_locals(self):
        return C.gq_qbx_locals(self.handle, self.n_ctr, self.p_qbx)

    def tree(self):
        return C.gq_tree_export(self.handle, self.n_ctr)

    def list(self, name):
        return C.gq_list_export(self.handle, name)

    def close(self):
        if self.handle:
            C.gq_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
