"""Python layer over the C ABI: torch tensors supply device memory and the
stream; every computation runs in libmfsem's HIP kernels.

Names follow the C entry points (mfsem_op_apply -> Operator.apply, ...).
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import torch

from . import _lib as L


# torch's current stream as a raw handle, without building a Stream object
# (that costs about 3 us per call, as much as a kernel launch)
_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream(stream=None, device=None):
    """The HIP stream to enqueue on: `stream`, else torch's current stream of
    device index `device` (default: the current device)."""
    if stream is not None:
        return C.c_void_p(stream.cuda_stream)
    if _raw_stream is not None:
        return C.c_void_p(_raw_stream(torch.cuda.current_device() if device is None else device))
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _workspace(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator returns 512-byte aligned blocks
    ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    assert ws.data_ptr() % 256 == 0
    return ws


def abi_version() -> int:
    return L.load().mfsem_abi_version()


# ----------------------------------------------------------------- meshes ---
class Box:
    """A structured box mesh generated on the device by mfsem_box_generate.

    elem_dof [n_elem][(p+1)^3] int32, xyz [n_dof][3] f64, fiber [n_dof][3] f64 or None."""

    def __init__(self, p, n, origin=(0.0, 0.0, 0.0), length=(1.0, 1.0, 1.0), shear_amp=0.0,
                 fiber=False, theta0=0.0, theta1=0.0, device="cuda"):
        lib = L.load()
        self.desc = L.BoxDesc(p=p, n=(C.c_int32 * 3)(*n), origin=(C.c_double * 3)(*origin),
                              length=(C.c_double * 3)(*length), shear_amp=shear_amp,
                              fiber=1 if fiber else 0, theta0=theta0, theta1=theta1)
        ne, nd = C.c_int64(), C.c_int64()
        L.check(lib.mfsem_box_counts(C.byref(self.desc), C.byref(ne), C.byref(nd)))
        self.p, self.n = p, tuple(n)
        self.n_elem, self.n_dof = ne.value, nd.value
        device = torch.device(device)
        if device.type == "cuda" and device.index is None:
            device = torch.device("cuda", torch.cuda.current_device())
        self.device = device
        P3 = (p + 1) ** 3
        self.elem_dof = torch.empty((self.n_elem, P3), dtype=torch.int32, device=device)
        self.xyz = torch.empty((self.n_dof, 3), dtype=torch.float64, device=device)
        self.fiber = (torch.empty((self.n_dof, 3), dtype=torch.float64, device=device)
                      if fiber else None)
        L.check(lib.mfsem_box_generate(C.byref(self.desc), _ptr(self.elem_dof), _ptr(self.xyz),
                                       _ptr(self.fiber), _stream()))
        self.spec = None

    @classmethod
    def from_spec(cls, spec, p=None, n=None, device="cuda"):
        """Mesh of a synth.BoxSpec (optionally with another degree / element count)."""
        b = cls(p if p is not None else spec.p, n if n is not None else spec.n, spec.origin,
                spec.length, spec.shear_amp, spec.fiber, spec.theta0, spec.theta1, device)
        b.spec = spec
        return b


def box_parents(n_fine, device="cuda"):
    """Octree parent element and child octant of every fine element."""
    ne = n_fine[0] * n_fine[1] * n_fine[2]
    parent = torch.empty(ne, dtype=torch.int32, device=device)
    child = torch.empty(ne, dtype=torch.int8, device=device)
    arr = (C.c_int32 * 3)(*n_fine)
    L.check(L.load().mfsem_box_parents(arr, _ptr(parent), _ptr(child), _stream()))
    return parent, child


# --------------------------------------------------------------- operator ---
class Operator:
    """A = alpha*M + K(sigma) on a mesh (mfsem_op_*).

    dofs: Box giving the DOF numbering (degree p); geometry: Box giving the map
    (defaults to `dofs`); xyz/fiber override the map's node data (e.g. jitter).
    geom: "auto" | "stored" | "onthefly" (mfsem_geometry): where the FP64
    stiffness apply takes G = W|J| J^-1 sigma J^-T from."""

    GEOM = {"auto": L.MFSEM_GEOM_AUTO, "stored": L.MFSEM_GEOM_STORED,
            "onthefly": L.MFSEM_GEOM_ONTHEFLY}

    def __init__(self, dofs: Box, geometry: Box | None = None, quad="gll", nq1d=0, sigma=None,
                 sigma_const=(1.0, 1.0, 1.0), batch=1, alpha=1.0, store_f64=True,
                 store_f32=False, xyz=None, fiber="geometry", sheet=None, structured=True,
                 geom="auto"):
        lib = L.load()
        geo = geometry or dofs
        self.dofs, self.geometry = dofs, geo
        self.device = dofs.device
        self.xyz = (xyz if xyz is not None else geo.xyz).contiguous()
        self.fiber = geo.fiber if isinstance(fiber, str) else fiber
        self.sheet = sheet
        if sigma is not None:
            sigma = torch.as_tensor(sigma, dtype=torch.float64, device=self.device).contiguous()
            batch = sigma.shape[0] if sigma.dim() == 3 else 1
            sigma = sigma.reshape(batch, dofs.n_elem, 3)
        self.sigma = sigma
        self.batch, self.p = batch, dofs.p
        self.n_dof, self.n_elem = dofs.n_dof, dofs.n_elem
        self.quad = quad
        q = nq1d if nq1d else dofs.p + 1
        self.q = q
        self.desc = L.OpDesc(
            p=dofs.p, quad=L.MFSEM_GLL if quad == "gll" else L.MFSEM_GAUSS, nq1d=q,
            n_elem=dofs.n_elem, n_dof=dofs.n_dof, elem_dof=dofs.elem_dof.data_ptr(),
            map_p=geo.p, map_elem_dof=geo.elem_dof.data_ptr(), n_map_nodes=geo.n_dof,
            map_xyz=self.xyz.data_ptr(), fiber=_ptr(self.fiber).value, sheet=_ptr(sheet).value,
            sigma=_ptr(sigma).value, sigma_const=(C.c_double * 3)(*sigma_const), batch=batch,
            alpha=alpha, store_f64=int(store_f64), store_f32=int(store_f32),
            lattice=(C.c_int32 * 3)(*(dofs.n if structured else (0, 0, 0))),
            geometry=self.GEOM[geom])
        nbytes = C.c_size_t()
        L.check(lib.mfsem_op_workspace_bytes(C.byref(self.desc), C.byref(nbytes)))
        self.ws = _workspace(nbytes.value, self.device)
        h = C.c_void_p()
        L.check(lib.mfsem_op_create(C.byref(self.desc), _ptr(self.ws), nbytes.value, _stream(),
                                    C.byref(h)))
        self.handle = h
        self.alpha = alpha
        self.store_f64, self.store_f32 = store_f64, store_f32
        self._lib = lib
        self._dev = self.ws.device.index

    @classmethod
    def from_spec(cls, spec, box=None, device="cuda", **kw):
        box = box or Box.from_spec(spec, device=device)
        args = dict(quad=spec.quad, nq1d=spec.q if spec.quad == "gauss" else 0,
                    sigma_const=spec.sigma, alpha=spec.alpha, sheet=spec_sheet(spec, box))
        args.update(kw)
        return cls(box, **args)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                L.load().mfsem_op_destroy(h)
            except Exception:  # at interpreter exit the binding may already be gone
                pass
            self.handle = None

    @staticmethod
    def _dt(t):
        if t.dtype == torch.float64:
            return L.MFSEM_F64
        if t.dtype == torch.float32:
            return L.MFSEM_F32
        raise TypeError("vectors must be float64 or float32")

    def _vec(self, x):
        if not (x.is_contiguous() and x.device == self.device and x.numel() == self.batch * self.n_dof):
            raise ValueError(f"expected a contiguous {self.batch}x{self.n_dof} vector on {self.device}")
        return x

    def apply(self, x, out=None, stream=None):
        """y = A x (mfsem_op_apply)."""
        x = self._vec(x)
        y = torch.empty_like(x) if out is None else self._vec(out)
        L.check(self._lib.mfsem_op_apply(self.handle, self._dt(x), x.data_ptr(), y.data_ptr(),
                                         _stream(stream, self._dev)))
        return y

    def apply_add(self, x, y, stream=None):
        """y += A x (mfsem_op_apply_add), one kernel launch."""
        x, y = self._vec(x), self._vec(y)
        L.check(self._lib.mfsem_op_apply_add(self.handle, self._dt(x), x.data_ptr(), y.data_ptr(),
                                             _stream(stream, self._dev)))
        return y

    def apply_mass(self, x, out=None):
        x = self._vec(x)
        y = torch.empty_like(x) if out is None else self._vec(out)
        L.check(L.load().mfsem_op_apply_mass(self.handle, self._dt(x), _ptr(x), _ptr(y), _stream()))
        return y

    def diagonal(self, dtype=torch.float64):
        d = torch.empty((self.batch, self.n_dof) if self.batch > 1 else (self.n_dof,),
                        dtype=dtype, device=self.device)
        L.check(L.load().mfsem_op_diagonal(self.handle, self._dt(d), _ptr(d), _stream()))
        return d

    def grad_sigma(self, u, w, scale=1.0):
        """g[b][e][c] = scale * w_b^T dA/dsigma_{e,c} u_b (mfsem_op_grad_sigma)."""
        u, w = self._vec(u.contiguous()), self._vec(w.contiguous())
        g = torch.empty((self.batch, self.n_elem, 3), dtype=torch.float64, device=self.device)
        L.check(L.load().mfsem_op_grad_sigma(self.handle, _ptr(u), _ptr(w), float(scale), _ptr(g),
                                             _stream()))
        return g

    def set_alpha(self, alpha):
        L.check(L.load().mfsem_op_set_alpha(self.handle, float(alpha)))
        self.alpha = alpha

    def set_sigma(self, sigma):
        s = torch.as_tensor(sigma, dtype=torch.float64, device=self.device).contiguous()
        L.check(L.load().mfsem_op_set_sigma(self.handle, _ptr(s), _stream()))
        self.sigma = s.reshape(self.batch, self.n_elem, 3)


# ----------------------------------------------------------- matrix-based ---
class CsrMatrix:
    """The operator assembled as a CSR matrix (mfsem_csr_*): the matrix-based
    path the paper compares the matrix-free one with.  pattern "element" stores
    every pair of nodes that share an element (collocation's zeros included, as
    a standard assembly does), "coupled" only the pairs that share a lattice
    coordinate (the entries collocation can make non-zero)."""

    PATTERNS = {"element": 0, "coupled": 1}

    def __init__(self, op: Operator, pattern: str = "element"):
        if pattern not in self.PATTERNS:
            raise ValueError(f"pattern must be one of {sorted(self.PATTERNS)}")
        lib = L.load()
        code = self.PATTERNS[pattern]
        nnz = C.c_int64()
        L.check(lib.mfsem_csr_nnz(op.handle, code, C.byref(nnz)))
        self.pattern = pattern
        self.n, self.nnz, self.device = op.n_dof, nnz.value, op.device
        self.row_ptr = torch.empty(self.n + 1, dtype=torch.int64, device=op.device)
        self.col = torch.empty(self.nnz, dtype=torch.int32, device=op.device)
        self.val = torch.empty(self.nnz, dtype=torch.float64, device=op.device)
        L.check(lib.mfsem_csr_assemble(op.handle, code, _ptr(self.row_ptr), _ptr(self.col),
                                       _ptr(self.val), _stream()))

    def apply(self, x, out=None):
        """y = A x (mfsem_csr_spmv)."""
        y = torch.empty_like(x) if out is None else out
        _pointwise(self.n, self.device, x, y)
        L.check(L.load().mfsem_csr_spmv(self.n, self.nnz, _ptr(self.row_ptr), _ptr(self.col),
                                        _ptr(self.val), _ptr(x), _ptr(y), _stream()))
        return y


# -------------------------------------------------------------- multigrid ---
class Multigrid:
    """V-cycle preconditioner over a list of level operators (mfsem_mg_*).

    transfers[l] = ("p",) or ("h", parent, child) links level l and l+1.
    coarse_degree: Chebyshev steps on the coarsest level (default 2 * degree).
    graphs: replay each (r, z) pair's V-cycle as one captured HIP graph (off by
    default: on MI355X the cycle is bound by the kernels, not by their launches,
    and replays measured the same as plain launches)."""

    def __init__(self, ops, transfers, degree=3, coarse_degree=None, lo=0.08, hi=1.2,
                 eig_iters=10, seed=12345, lambda_max=None, precision=torch.float64,
                 graphs=False):
        lib = L.load()
        self.ops = list(ops)
        self.batch = self.ops[0].batch
        nl = len(self.ops)
        self._ops_arr = (C.c_void_p * nl)(*[o.handle.value for o in self.ops])
        trs = (L.TransferDesc * max(1, nl - 1))()
        self._keep = []
        for i, t in enumerate(transfers):
            if t[0] == "p":
                trs[i] = L.TransferDesc(kind=L.MFSEM_TRANSFER_P, parent=None, child=None)
            else:
                parent, child = t[1], t[2]
                nf = self.ops[i].n_elem
                if (parent.dtype != torch.int32 or child.dtype != torch.int8 or not parent.is_cuda
                        or not child.is_cuda or parent.numel() != nf or child.numel() != nf
                        or not parent.is_contiguous() or not child.is_contiguous()):
                    raise ValueError(f"h-transfer {i}: parent (int32) and child (int8) need "
                                     f"{nf} contiguous CUDA entries")
                self._keep += [parent, child]
                trs[i] = L.TransferDesc(kind=L.MFSEM_TRANSFER_H, parent=parent.data_ptr(),
                                        child=child.data_ptr())
        self._trs = trs
        self.transfers = list(transfers)
        lam = None
        if lambda_max is not None:
            vals = [float(v) for v in torch.as_tensor(lambda_max, dtype=torch.float64).reshape(-1)]
            lam = (C.c_double * len(vals))(*vals)
        self.precision = precision
        self.desc = L.MgDesc(n_levels=nl, ops=self._ops_arr, transfers=trs, degree=degree,
                             coarse_degree=coarse_degree or 2 * degree, lo_frac=lo, hi_frac=hi,
                             eig_iters=eig_iters, eig_seed=seed, lambda_max=lam,
                             precision=L.MFSEM_F64 if precision == torch.float64 else L.MFSEM_F32,
                             graphs=int(graphs))
        nbytes = C.c_size_t()
        L.check(lib.mfsem_mg_workspace_bytes(C.byref(self.desc), C.byref(nbytes)))
        self.ws = _workspace(nbytes.value, self.ops[0].device)
        h = C.c_void_p()
        L.check(lib.mfsem_mg_create(C.byref(self.desc), _ptr(self.ws), nbytes.value, _stream(),
                                    C.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                L.load().mfsem_mg_destroy(h)
            except Exception:  # at interpreter exit the binding may already be gone
                pass
            self.handle = None

    def vcycle(self, r, out=None):
        z = torch.empty_like(r) if out is None else out
        L.check(L.load().mfsem_mg_vcycle(self.handle, _ptr(r), _ptr(z), _stream()))
        return z

    def _check_vec(self, v, level):
        if v.dtype != self.precision or not v.is_cuda or not v.is_contiguous():
            raise ValueError(f"expected a contiguous {self.precision} CUDA tensor")
        if v.numel() != self.batch * self.ops[level].n_dof:
            raise ValueError(f"expected {self.batch} x {self.ops[level].n_dof} values")

    def prolong(self, level, xc):
        """Fine-level vector P xc (mfsem_mg_transfer, direction 0)."""
        self._check_vec(xc, level + 1)
        xf = torch.empty((self.batch, self.ops[level].n_dof) if self.batch > 1 else
                         (self.ops[level].n_dof,), dtype=xc.dtype, device=xc.device)
        L.check(L.load().mfsem_mg_transfer(self.handle, level, 0, _ptr(xc), _ptr(xf), _stream()))
        return xf

    def restrict(self, level, rf):
        """Coarse-level vector P^T rf (mfsem_mg_transfer, direction 1)."""
        self._check_vec(rf, level)
        rc = torch.empty((self.batch, self.ops[level + 1].n_dof) if self.batch > 1 else
                         (self.ops[level + 1].n_dof,), dtype=rf.dtype, device=rf.device)
        L.check(L.load().mfsem_mg_transfer(self.handle, level, 1, _ptr(rf), _ptr(rc), _stream()))
        return rc

    def lambdas(self):
        n = len(self.ops) * self.batch
        arr = (C.c_double * n)()
        L.check(L.load().mfsem_mg_lambdas(self.handle, arr))
        return torch.tensor(list(arr), dtype=torch.float64).reshape(len(self.ops), self.batch)


def spec_sheet(spec, box):
    """The sheet field of a spec with a sheet (the in-plane normal of the box's
    fiber, (-a_y, a_x, 0)), or None."""
    if not getattr(spec, "sheet", False):
        return None
    f = box.fiber
    return torch.stack([-f[:, 1], f[:, 0], torch.zeros_like(f[:, 0])], dim=1).contiguous()


def hierarchy(spec, fine_box: Box | None = None, coarsening=(("p", 2), ("p", 1)),
              precision=torch.float64, device="cuda", sigma=None, xyz=None, structured=True,
              **mg_kw):
    """Operators and multigrid for a synth.BoxSpec.

    coarsening: sequence of ("p", degree) and ("h",) steps from the finest level.
    p-levels keep the geometry map of the level they coarsen; h-levels build the
    octree-coarser box from the same recipe.  Levels below the finest use GLL
    quadrature (SEM-NI) whatever the finest level's rule: the preconditioner
    only needs a spectrally equivalent operator, and the collocated one is the
    cheapest.  structured=False builds every level as a general mesh (element
    kernels and element transfers)."""
    fine_box = fine_box or Box.from_spec(spec, device=device)
    store = dict(store_f64=True, store_f32=(precision == torch.float32))
    kw = dict(sigma_const=spec.sigma, alpha=spec.alpha, sigma=sigma, structured=structured)
    ops = [Operator(fine_box, quad=spec.quad, nq1d=spec.q if spec.quad == "gauss" else 0,
                    xyz=xyz, sheet=spec_sheet(spec, fine_box), **store, **kw)]
    boxes = [fine_box]
    geo_box, geo_xyz, n = fine_box, xyz, spec.n
    amp = spec.shear_amp
    transfers = []
    for step in coarsening:
        prev = ops[-1]
        if step[0] == "p":
            pc = step[1]
            dofs = Box(pc, n, spec.origin, spec.length, amp, spec.fiber, spec.theta0,
                       spec.theta1, device)
            ops.append(Operator(dofs, geometry=geo_box, xyz=geo_xyz,
                                sheet=spec_sheet(spec, geo_box), **store, **kw))
            transfers.append(("p",))
        else:
            if sigma is not None:
                raise ValueError("per-element sigma with h-coarsening is not supported")
            nc = tuple(k // 2 for k in n)
            parent, child = box_parents(n, device=device)
            # the shear amplitude is relative to the element edge: halve it so the
            # coarse mesh samples the same displacement field
            amp = amp / 2
            geo_box = Box(prev.p, nc, spec.origin, spec.length, amp, spec.fiber, spec.theta0,
                          spec.theta1, device)
            geo_xyz = None
            ops.append(Operator(geo_box, sheet=spec_sheet(spec, geo_box), **store, **kw))
            transfers.append(("h", parent, child))
            n = nc
            dofs = geo_box
        boxes.append(dofs)
    mg = Multigrid(ops, transfers, precision=precision, **mg_kw)
    mg.boxes = boxes
    return ops, mg


# ------------------------------------------------------- node placement ---
def place_nodes(kind: str, p: int, elem_dof, xyz, fiber, elem, loc, pc: int = 0):
    """Coordinates (and fibers) of new nodes from a parent mesh's degree-p map
    (mfsem_mesh_refine_nodes for kind "refine", mfsem_mesh_degree_nodes with
    degree pc for kind "degree"): new node g at point loc[g] of element
    elem[g]'s reference lattice.  Device tensors in, device tensors out."""
    if kind not in ("refine", "degree"):
        raise ValueError("kind must be 'refine' or 'degree'")
    for a, dt in ((elem_dof, torch.int32), (xyz, torch.float64), (elem, torch.int32),
                  (loc, torch.int32)):
        if a.dtype != dt or not a.is_cuda or not a.is_contiguous():
            raise ValueError(f"expected a contiguous {dt} CUDA tensor")
    if fiber is not None and (fiber.dtype != torch.float64 or fiber.shape != xyz.shape
                              or not fiber.is_contiguous()):
        raise ValueError("fiber must be a contiguous float64 tensor shaped like xyz")
    if elem.numel() != loc.numel():
        raise ValueError("elem and loc must have one entry per new node")
    n_new = elem.numel()
    out = torch.empty((n_new, 3), dtype=torch.float64, device=xyz.device)
    fout = None if fiber is None else torch.empty_like(out)
    lib = L.load()
    args = (p, elem_dof.shape[0], _ptr(elem_dof), xyz.shape[0], _ptr(xyz), _ptr(fiber))
    tail = (n_new, _ptr(elem), _ptr(loc), _ptr(out), _ptr(fout), _stream())
    if kind == "refine":
        L.check(lib.mfsem_mesh_refine_nodes(*args, *tail))
    else:
        L.check(lib.mfsem_mesh_degree_nodes(*args, pc, *tail))
    return out, fout


# -------------------------------------------------------------------- PCG ---
@dataclass
class SolveInfo:
    iters: list
    status: list
    r0_norm: list
    r_norm: list
    b_norm: list


def pcg(op: Operator, b, x0=None, mg: Multigrid | None = None, rtol=1e-10, atol=0.0,
        max_it=1000, flexible=None, check=True):
    """Solve A x = b by (P)CG (mfsem_pcg).  Returns (x, SolveInfo)."""
    lib = L.load()
    b = op._vec(b.contiguous())
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    if flexible is None:
        flexible = mg is not None and mg.precision == torch.float32
    nbytes = C.c_size_t()
    L.check(lib.mfsem_pcg_workspace_bytes(op.handle, mg.handle if mg else None, C.byref(nbytes)))
    ws = _workspace(nbytes.value, op.device)
    opts = L.SolveOpts(rtol=rtol, atol=atol, max_it=max_it, flexible=int(flexible))
    infos = (L.SolveInfo * op.batch)()
    st = lib.mfsem_pcg(op.handle, mg.handle if mg else None, _ptr(b), _ptr(x), C.byref(opts),
                       infos, _ptr(ws), nbytes.value, _stream())
    info = SolveInfo([i.iters for i in infos], [i.status for i in infos],
                     [i.r0_norm for i in infos], [i.r_norm for i in infos],
                     [i.b_norm for i in infos])
    if check and st != L.MFSEM_OK:
        L.check(st)
    return x, info


# ------------------------------------------------------------------ ionic ---
def _ap_params(params: dict):
    return L.APParams(**{k: float(params[k]) for k in ("k", "a", "eps0", "mu1", "mu2", "v_rest",
                                                       "v_amp", "t_scale")})


def _pointwise(n, device, *arrays):
    """The pointwise kernels index every array with the same n FP64 entries."""
    for a in arrays:
        if a is None:
            continue
        if not (a.dtype == torch.float64 and a.is_contiguous() and a.numel() == n
                and a.device == device):
            raise ValueError(f"expected contiguous float64 arrays of {n} entries on {device}")


def ap_imex_rhs(V, w, mass_diag, dt, chi, cm, params: dict, i_stim=None, out=None):
    """b and the updated gate w for one IMEX step (mfsem_ap_imex_rhs)."""
    b = torch.empty_like(V) if out is None else out
    _pointwise(V.numel(), V.device, V, w, mass_diag, i_stim, b)
    prm = _ap_params(params)
    L.check(L.load().mfsem_ap_imex_rhs(V.numel(), dt, chi, cm, C.byref(prm), _ptr(V), _ptr(w),
                                       _ptr(i_stim), _ptr(mass_diag), _ptr(b), _stream()))
    return b


def ap_bdf2_rhs(V, V_old, w, w_old, mass_diag, dt, chi, cm, params: dict, i_stim=None,
                out=None):
    """b of the BDF2 step; w_old <- w, w <- w^{n+1} (mfsem_ap_bdf2_rhs)."""
    b = torch.empty_like(V) if out is None else out
    _pointwise(V.numel(), V.device, V, V_old, w, w_old, mass_diag, i_stim, b)
    prm = _ap_params(params)
    L.check(L.load().mfsem_ap_bdf2_rhs(V.numel(), dt, chi, cm, C.byref(prm), _ptr(V),
                                       _ptr(V_old), _ptr(w), _ptr(w_old), _ptr(i_stim),
                                       _ptr(mass_diag), _ptr(b), _stream()))
    return b


def activation_update(V, V_old, t, dt, act=None, rate=None, v_cross=0.0, cross=None):
    """Running activation times after a step from V_old (at t - dt) to V (at t):
    act, rate take the step's midpoint and |dV/dt| where it is the steepest
    so far; cross records the first upward crossing of v_cross
    (mfsem_activation_update).  Updated in place."""
    _pointwise(V.numel(), V.device, V, V_old, act, rate, cross)
    L.check(L.load().mfsem_activation_update(V.numel(), float(t), float(dt), _ptr(V),
                                             _ptr(V_old), _ptr(act), _ptr(rate), float(v_cross),
                                             _ptr(cross), _stream()))


def extrapolate(v, v_old, out=None):
    """2 v - v_old, the initial guess of the next implicit solve (mfsem_extrapolate)."""
    y = torch.empty_like(v) if out is None else out
    _pointwise(v.numel(), v.device, v, v_old, y)
    L.check(L.load().mfsem_extrapolate(v.numel(), _ptr(v), _ptr(v_old), _ptr(y), _stream()))
    return y
