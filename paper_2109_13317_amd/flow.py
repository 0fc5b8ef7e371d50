"""Python face of libpffrg: same names as the C ABI, argument marshalling only.

Device memory and streams come from PyTorch (float64 CUDA tensors on ROCm);
every step of the flow runs in the library's HIP kernels.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from .lattice import LatticeTables, build_tables


def _dptr(t: torch.Tensor) -> ctypes.c_void_p:
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 tensor on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def _lattice_struct(t: LatticeTables):
    """(pffrg_lattice, arrays it points into: keep them alive for the call)."""
    keep = [np.ascontiguousarray(a, dtype=np.int32) for a in (t.swap, t.mult, t.rpa_off, t.rpa_ka,
                                                              t.rpa_kb, t.rpa_cnt)]
    # an XYZ model's coupling triples go to pffrg_create_xyz and a general
    # model's matrices to pffrg_create_tri; the lattice struct then carries a
    # component of them, which it does not read
    coup = t.coupling.reshape(len(t.coupling), -1)[:, 0]
    keep += [np.ascontiguousarray(coup, dtype=np.float64),
             np.ascontiguousarray(t.site_pair, dtype=np.int32),
             np.ascontiguousarray(t.site_pos, dtype=np.float64),
             np.ascontiguousarray(t.basis_pos, dtype=np.float64)]
    ptr = [ctypes.c_void_p(a.ctypes.data) for a in keep]
    lat = _lib.Lattice(t.n_pairs, ptr[0], ptr[1], ptr[2], ptr[3], ptr[4], ptr[5], ptr[6],
                       t.n_basis, t.n_sites_total, ptr[7], ptr[8], ptr[9])
    return lat, keep


def _spin_rot_struct(t: LatticeTables):
    """(pffrg_spin_rot or None, arrays it points into) for tables reduced with
    spin permutations: each rotation as its rows, row a holding sign(v) in
    column |v| - 1."""
    if t.rot is None:
        return None, []
    rows = np.zeros((len(t.rot), 3), dtype=np.int32)
    for r, W in enumerate(np.asarray(t.rot)):
        for a in range(3):
            col = int(np.argmax(np.abs(W[a])))
            rows[r, a] = int(np.sign(W[a, col])) * (col + 1)
    keep = [np.ascontiguousarray(a, dtype=np.int32) for a in (rows, t.swap_rot, t.rpa_rot_a, t.rpa_rot_b, t.site_rot)]
    ptr = [ctypes.c_void_p(a.ctypes.data) for a in keep]
    return _lib.SpinRot(len(t.rot), *ptr), keep


class Context:
    """A ``pffrg_ctx``: one lattice model on one frequency mesh.  Tables of a
    Heisenberg model give an SU(2) context (two strains, spin and density);
    tables of an XYZ model (coupling triples) an XYZ context (four strains:
    x, y, z, density); tables of a general model (3x3 coupling matrices) a
    TRI context (sixteen strains Gamma^{mu nu}, index 4 mu + nu, FP64)."""

    def __init__(self, tables: LatticeTables, mesh, precision: str = "fp64", stream=None):
        self.lib = _lib.load()
        self.tables = tables
        self.precision = precision
        self.mesh = np.ascontiguousarray(mesh, dtype=np.float64)
        self.nf = len(self.mesh)
        self.ns = tables.n_pairs
        self.symmetry = {1: "su2", 2: "xyz", 3: "tri"}[tables.coupling.ndim]
        if tables.rot is not None and self.symmetry != "tri":
            raise ValueError("the SU(2) and XYZ kernels take tables without spin rotations: build them with "
                             "spin_permutations=False, or run the model as a general one (3x3 matrices, TRI)")
        self.nc = {"su2": 2, "xyz": 4, "tri": 16}[self.symmetry]
        lat, keep = _lattice_struct(tables)
        msh = _lib.Mesh(self.nf, ctypes.c_void_p(self.mesh.ctypes.data))
        prec = {"fp64": _lib.FP64, "fp32": _lib.FP32}[precision]
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        if self.symmetry == "xyz":
            c3 = np.ascontiguousarray(np.asarray(tables.coupling, dtype=np.float64).T)     # [3][ns]
            _lib.check(self.lib.pffrg_create_xyz(ctypes.byref(lat), ctypes.c_void_p(c3.ctypes.data),
                                                 ctypes.byref(msh), prec, ctypes.c_void_p(stream.cuda_stream),
                                                 ctypes.byref(h)))
        elif self.symmetry == "tri":
            c9 = np.ascontiguousarray(tables.coupling, dtype=np.float64)                   # [ns][3][3]
            srot, keep_rot = _spin_rot_struct(tables)
            _lib.check(self.lib.pffrg_create_tri(ctypes.byref(lat), ctypes.c_void_p(c9.ctypes.data),
                                                 ctypes.byref(srot) if srot is not None else None,
                                                 ctypes.byref(msh), prec, ctypes.c_void_p(stream.cuda_stream),
                                                 ctypes.byref(h)))
        else:
            _lib.check(self.lib.pffrg_create(ctypes.byref(lat), ctypes.byref(msh), prec,
                                             ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.handle = h
        n = ctypes.c_size_t()
        _lib.check(self.lib.pffrg_state_size(self.handle, ctypes.byref(n)))
        self.size = int(n.value)
        self.n_su = self.nf * (self.nf + 1) // 2
        self.vsize = self.n_su * self.nf * self.ns

    @classmethod
    def from_model(cls, model, lattice_range, mesh, **kw):
        return cls(build_tables(model, lattice_range), mesh, **kw)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.check(self.lib.pffrg_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ state --
    def new_state(self) -> torch.Tensor:
        return torch.empty(self.size, dtype=torch.float64, device="cuda")

    def split(self, x: torch.Tensor):
        """Views (sig[nf], strain 0, strain 1, ...), each strain [n_su, nf, ns]:
        SU(2) (sig, Gs, Gd), XYZ (sig, Gx, Gy, Gz, Gd), TRI (sig, G^{00},
        G^{01}, ..., G^{33})."""
        nf, v = self.nf, self.vsize
        return (x[:nf],) + tuple(x[nf + c * v:nf + (c + 1) * v].view(self.n_su, nf, self.ns)
                                 for c in range(self.nc))

    def init_state(self, x: torch.Tensor | None = None) -> torch.Tensor:
        x = self.new_state() if x is None else x
        _lib.check(self.lib.pffrg_init_state(self.handle, _dptr(x)))
        return x

    # -------------------------------------------------------------- flow --
    def rhs(self, lam: float, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        out = self.new_state() if out is None else out
        _lib.check(self.lib.pffrg_rhs(self.handle, float(lam), _dptr(x), _dptr(out)))
        return out

    def sigma_rhs(self, lam: float, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        out = torch.empty(self.nf, dtype=torch.float64, device="cuda") if out is None else out
        _lib.check(self.lib.pffrg_sigma_rhs(self.handle, float(lam), _dptr(x), _dptr(out)))
        return out

    def step(self, scheme: str, lam0: float, lam1: float, x: torch.Tensor) -> torch.Tensor:
        sc = {"euler": _lib.EULER, "rk4": _lib.RK4}[scheme]
        _lib.check(self.lib.pffrg_step(self.handle, sc, float(lam0), float(lam1), _dptr(x)))
        return x

    def flow(self, x: torch.Tensor, *, schedule=None, scheme: str = "rk4", lam_start=None,
             lam_stop=None, rtol=1e-6, atol=1e-10, h0=0.05, hmin=1e-8, max_steps=0,
             kpoints: torch.Tensor | None = None, observer=None, resume=None) -> int:
        """Integrate x in place; observer(lam, chi_pairs[2, ns], chi_k or None)
        receives torch views of the library's device buffers (copy to keep).
        resume=(log_lambda, ladder) continues an adaptive flow from a position
        that position() reported (lam_start is then ignored)."""
        o = _lib.FlowOpts()
        o.scheme = {"euler": _lib.EULER, "rk4": _lib.RK4, "dopri54": _lib.DOPRI54}[scheme]
        sched = None
        if scheme in ("euler", "rk4"):
            sched = np.ascontiguousarray(schedule, dtype=np.float64)
            o.n_lambda = len(sched)
            o.lambdas = ctypes.c_void_p(sched.ctypes.data)
        else:
            o.lam_start = float(lam_start) if lam_start is not None else 0.0
            o.lam_stop = float(lam_stop)
            if resume is not None:
                o.resume, o.resume_log_lambda, o.resume_ladder = 1, float(resume[0]), int(resume[1])
        o.rtol, o.atol, o.h0, o.hmin, o.max_steps = rtol, atol, h0, hmin, int(max_steps)
        chik = None
        if kpoints is not None:
            kp = kpoints.contiguous()
            chik = torch.empty(kp.shape[0], dtype=torch.float64, device="cuda")
            o.n_k, o.d_k, o.d_chi_k = int(kp.shape[0]), _dptr(kp), _dptr(chik)
        ns = self.ns

        def _cb(lam, dchi, dchik, _user):
            if observer is None:
                return 0
            chi = _wrap(dchi, self.nc * ns).view(self.nc, ns)
            ck = chik if dchik else None
            return int(bool(observer(lam, chi, ck)))

        cb = _lib.OBSERVER(_cb) if observer is not None else _lib.OBSERVER()
        nsteps = ctypes.c_int()
        _lib.check(self.lib.pffrg_flow(self.handle, ctypes.byref(o), _dptr(x), cb, None,
                                       ctypes.byref(nsteps)))
        del sched
        return int(nsteps.value)

    def position(self) -> tuple[float, float, int]:
        """(lambda, ln lambda, ladder index) of the last accepted flow step:
        the adaptive controller's step index, or for fixed schedules the index
        of the accepted cutoff in the schedule."""
        lam, ll, lad = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        _lib.check(self.lib.pffrg_flow_position(self.handle, ctypes.byref(lam), ctypes.byref(ll),
                                                ctypes.byref(lad)))
        return lam.value, ll.value, lad.value

    # ------------------------------------------------------ reverse mode --
    def init_state_from(self, coupling, x: torch.Tensor | None = None) -> torch.Tensor:
        """Initial condition for per-pair couplings (device or host array)."""
        x = self.new_state() if x is None else x
        cp = torch.as_tensor(np.asarray(coupling, dtype=np.float64) if not torch.is_tensor(coupling)
                             else coupling, dtype=torch.float64).cuda().contiguous()
        _lib.check(self.lib.pffrg_init_state_from(self.handle, _dptr(cp), _dptr(x)))
        return x

    def rhs_vjp(self, lam: float, x: torch.Tensor, cot: torch.Tensor, out: torch.Tensor | None = None):
        out = self.new_state() if out is None else out
        _lib.check(self.lib.pffrg_rhs_vjp(self.handle, float(lam), _dptr(x), _dptr(cot), _dptr(out)))
        return out

    def chi_vjp(self, lam: float, x: torch.Tensor, cot_chi: torch.Tensor, out: torch.Tensor | None = None):
        out = self.new_state() if out is None else out
        _lib.check(self.lib.pffrg_chi_vjp(self.handle, float(lam), _dptr(x), _dptr(cot_chi.contiguous().view(-1)),
                                          _dptr(out)))
        return out

    def chi_k_vjp(self, cot_chi_k: torch.Tensor, kpoints: torch.Tensor) -> torch.Tensor:
        kp = kpoints.contiguous()
        out = torch.empty(2 * self.ns, dtype=torch.float64, device="cuda")
        _lib.check(self.lib.pffrg_chi_k_vjp(self.handle, _dptr(cot_chi_k.contiguous()), int(kp.shape[0]),
                                            _dptr(kp), _dptr(out)))
        return out.view(2, self.ns)

    def flow_checkpoints(self, x: torch.Tensor, schedule) -> torch.Tensor:
        """RK4 along schedule in place; returns the checkpoints [steps, size]."""
        sched = np.ascontiguousarray(schedule, dtype=np.float64)
        ck = torch.empty((len(sched) - 1, self.size), dtype=torch.float64, device="cuda")
        _lib.check(self.lib.pffrg_flow_checkpoints(self.handle, len(sched), ctypes.c_void_p(sched.ctypes.data),
                                                   _dptr(x), _dptr(ck)))
        return ck

    def flow_vjp(self, schedule, checkpoints: torch.Tensor, cot: torch.Tensor) -> torch.Tensor:
        """cot: final-state cotangent, replaced by the initial-state one;
        returns d/d coupling per pair."""
        sched = np.ascontiguousarray(schedule, dtype=np.float64)
        dcp = torch.empty(self.ns, dtype=torch.float64, device="cuda")
        _lib.check(self.lib.pffrg_flow_vjp(self.handle, len(sched), ctypes.c_void_p(sched.ctypes.data),
                                           _dptr(checkpoints), _dptr(cot), _dptr(dcp)))
        return dcp

    # --------------------------------------------------------- profiling --
    _KERNELS = {"sigma": _lib.K_SIGMA, "tables": _lib.K_TABLES, "vertex": _lib.K_VERTEX,
                "vertex_s": _lib.K_VERTEX_S, "vertex_u": _lib.K_VERTEX_U, "vertex_t": _lib.K_VERTEX_T,
                "vertex_stu": _lib.K_VERTEX_STU}

    def set_vertex_mode(self, mode: str):
        """How the vertex channels are launched: 'auto' (default), 'one_launch',
        'separate' or 'concurrent' (pffrg_set_vertex_mode; same results bitwise)."""
        _lib.check(self.lib.pffrg_set_vertex_mode(self.handle, _lib.VERTEX_MODES[mode]))

    def set_profiling(self, on: bool, kernels=None):
        """Record kernel durations with HIP events: all timed kernels, or only
        the named ones (names as in profile_read); False turns it off.
        Timing 'vertex_s', 'vertex_u' or 'vertex_t' (also implied by all)
        runs the three channels as separate launches (same results bitwise);
        otherwise they run in the context's vertex mode ('vertex_stu' is the
        one-launch form, 'vertex' spans any form)."""
        if kernels is None or not on:
            _lib.check(self.lib.pffrg_set_profiling(self.handle, int(bool(on))))
        else:
            mask = 0
            for k in kernels:
                mask |= 1 << self._KERNELS[k]
            _lib.check(self.lib.pffrg_set_profiling_mask(self.handle, mask))

    def profile_read(self, kernel: str):
        """(total_ms, launches) of 'sigma', 'tables', 'vertex' (all vertex
        launches), 'vertex_stu', 'vertex_s', 'vertex_u' or 'vertex_t' since
        profiling began."""
        kid = self._KERNELS[kernel]
        ms, n = ctypes.c_double(), ctypes.c_int()
        _lib.check(self.lib.pffrg_profile_read(self.handle, kid, ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)

    # ------------------------------------------------------- observables --
    def chi(self, lam: float, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """[strains, ns] per reduced pair: SU(2) chi^{zz}, chi^{00}; XYZ chi^{xx},
        chi^{yy}, chi^{zz}, chi^{00}; TRI the real parts of chi^{mu nu} at
        4 mu + nu."""
        out = torch.empty(self.nc * self.ns, dtype=torch.float64, device="cuda") if out is None else out
        _lib.check(self.lib.pffrg_chi(self.handle, float(lam), _dptr(x), _dptr(out)))
        return out.view(self.nc, self.ns)

    def chi_k(self, chi: torch.Tensor, kpoints: torch.Tensor, out: torch.Tensor | None = None):
        kp = kpoints.contiguous()
        out = torch.empty(kp.shape[0], dtype=torch.float64, device="cuda") if out is None else out
        _lib.check(self.lib.pffrg_chi_k(self.handle, _dptr(chi.contiguous()), int(kp.shape[0]),
                                        _dptr(kp), _dptr(out)))
        return out

    def chi_sites(self, chi: torch.Tensor) -> torch.Tensor:
        """chi per reduced pair spread onto [strains, n_basis, n_sites_total]
        (the layout of the paper's observable files; NaN past a basis site's
        sites in range)."""
        nb, nst = self.tables.n_basis, self.tables.n_sites_total
        out = torch.empty(self.nc * nb * nst, dtype=torch.float64, device="cuda")
        _lib.check(self.lib.pffrg_chi_sites(self.handle, _dptr(chi.contiguous()), _dptr(out)))
        return out.view(self.nc, nb, nst)


class ChiAdjoint(torch.autograd.Function):
    """chi(k) at the end of an RK4 flow as a differentiable function of the
    couplings J (one per coupling shell): the initial condition takes the
    per-pair couplings design @ J; the backward pass is the library's
    discrete adjoint (checkpointed steps).

    forward(J, ctx, design [ns, nJ], schedule, kpoints [nk, 3]) -> chi(k) [nk]
    """

    @staticmethod
    def forward(fctx, J, ctx, design, schedule, kpoints):
        Jn = J.detach().cpu().numpy().astype(np.float64)
        coupling = np.asarray(design, dtype=np.float64) @ Jn
        x = ctx.init_state_from(coupling)
        ck = ctx.flow_checkpoints(x, schedule)
        lam = float(schedule[-1])
        chi = ctx.chi(lam, x)
        kp = kpoints.to(device="cuda", dtype=torch.float64).contiguous()
        out = ctx.chi_k(chi, kp)
        fctx.save_for_backward(J)
        fctx.stash = (ctx, np.asarray(design, dtype=np.float64), np.asarray(schedule, dtype=np.float64), x, ck, kp)
        return out.to(J.device)

    @staticmethod
    def backward(fctx, grad):
        (J,) = fctx.saved_tensors
        ctx, design, schedule, x, ck, kp = fctx.stash
        g = grad.detach().to(device="cuda", dtype=torch.float64).contiguous()
        cchi = ctx.chi_k_vjp(g, kp)
        cot = ctx.chi_vjp(float(schedule[-1]), x, cchi)
        dcp = ctx.flow_vjp(schedule, ck, cot)
        dJ = design.T @ dcp.cpu().numpy()
        return torch.as_tensor(dJ, dtype=J.dtype, device=J.device), None, None, None, None


class Batch:
    """A ``pffrg_batch``: many lattice models on one mesh, advanced in lockstep.

    The batch state is one float64 tensor; ``offsets[p]`` is where point p's
    state (single-flow layout) begins."""

    def __init__(self, tables: list[LatticeTables], mesh, precision: str = "fp32", stream=None):
        self.lib = _lib.load()
        self.tables = list(tables)
        self.precision = precision
        self.mesh = np.ascontiguousarray(mesh, dtype=np.float64)
        self.nf = len(self.mesh)
        self.n_points = len(self.tables)
        self.ns = [t.n_pairs for t in self.tables]
        structs, keep = [], []
        for t in self.tables:
            lat, k = _lattice_struct(t)
            structs.append(lat)
            keep.append(k)
        arr = (ctypes.POINTER(_lib.Lattice) * self.n_points)(*[ctypes.pointer(s) for s in structs])
        msh = _lib.Mesh(self.nf, ctypes.c_void_p(self.mesh.ctypes.data))
        prec = {"fp64": _lib.FP64, "fp32": _lib.FP32}[precision]
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        _lib.check(self.lib.pffrg_batch_create(self.n_points, arr, ctypes.byref(msh), prec,
                                               ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.handle = h
        off = (ctypes.c_size_t * (self.n_points + 1))()
        _lib.check(self.lib.pffrg_batch_state_offsets(self.handle, off))
        self.offsets = [int(v) for v in off]
        self.size = self.offsets[-1]
        self.chi_offsets = list(np.concatenate([[0], np.cumsum([2 * n for n in self.ns])]))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.check(self.lib.pffrg_batch_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_state(self) -> torch.Tensor:
        return torch.empty(self.size, dtype=torch.float64, device="cuda")

    def point(self, x: torch.Tensor, p: int) -> torch.Tensor:
        """View of point p's state inside a batch state."""
        return x[self.offsets[p]:self.offsets[p + 1]]

    def init_state(self, x: torch.Tensor | None = None) -> torch.Tensor:
        x = self.new_state() if x is None else x
        _lib.check(self.lib.pffrg_batch_init_state(self.handle, _dptr(x)))
        return x

    def rhs(self, lam: float, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        out = self.new_state() if out is None else out
        _lib.check(self.lib.pffrg_batch_rhs(self.handle, float(lam), _dptr(x), _dptr(out)))
        return out

    def flow(self, x: torch.Tensor, schedule, use_graph: bool = True) -> list[bool]:
        """Lockstep RK4 along schedule, in place; per-point finiteness."""
        sched = np.ascontiguousarray(schedule, dtype=np.float64)
        ok = (ctypes.c_int * self.n_points)()
        _lib.check(self.lib.pffrg_batch_flow(self.handle, len(sched), ctypes.c_void_p(sched.ctypes.data),
                                             _dptr(x), int(bool(use_graph)), ok))
        return [bool(v) for v in ok]

    def chi(self, lam: float, x: torch.Tensor) -> list[torch.Tensor]:
        """[2, ns_p] per point."""
        out = torch.empty(int(self.chi_offsets[-1]), dtype=torch.float64, device="cuda")
        _lib.check(self.lib.pffrg_batch_chi(self.handle, float(lam), _dptr(x), _dptr(out)))
        return [out[self.chi_offsets[p]:self.chi_offsets[p + 1]].view(2, self.ns[p])
                for p in range(self.n_points)]

    def chi_k(self, p: int, chi: torch.Tensor, kpoints: torch.Tensor) -> torch.Tensor:
        kp = kpoints.contiguous()
        out = torch.empty(kp.shape[0], dtype=torch.float64, device="cuda")
        _lib.check(self.lib.pffrg_batch_chi_k(self.handle, int(p), _dptr(chi.contiguous().view(-1)),
                                              int(kp.shape[0]), _dptr(kp), _dptr(out)))
        return out

    def tune(self, lam: float, x: torch.Tensor) -> tuple[int, int, int]:
        """Autotune the vertex launch; (workgroups per XCD, tile order, split)."""
        per, order, split = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _lib.check(self.lib.pffrg_batch_tune(self.handle, float(lam), _dptr(x), ctypes.byref(per),
                                             ctypes.byref(order), ctypes.byref(split)))
        return int(per.value), int(order.value), int(split.value)

    def set_launch(self, per: int, order: int, split: int = 0):
        _lib.check(self.lib.pffrg_batch_set_launch(self.handle, int(per), int(order), int(split)))

    def set_profiling(self, on: bool):
        _lib.check(self.lib.pffrg_batch_set_profiling(self.handle, int(bool(on))))

    def profile_read(self):
        ms, n = ctypes.c_double(), ctypes.c_int()
        _lib.check(self.lib.pffrg_batch_profile_read(self.handle, ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)


class _Peaks(ctypes.Structure):
    _fields_ = [("fp64_fma_tflops", ctypes.c_double), ("fp32_fma_tflops", ctypes.c_double),
                ("hbm_copy_gbs", ctypes.c_double), ("l1_load_tbs", ctypes.c_double),
                ("l1_load_2row_tbs", ctypes.c_double), ("lds_read_tbs", ctypes.c_double)]


def measure_peaks(stream=None) -> dict:
    """Measured FP64 / FP32 vector FMA throughput (TFLOP/s), device-copy
    bandwidth (GB/s) and the 16-byte-per-lane load rates from L1 and LDS
    (TB/s) of the current device (pffrg_measure_peaks)."""
    lib = _lib.load()
    stream = torch.cuda.current_stream() if stream is None else stream
    out = _Peaks()
    _lib.check(lib.pffrg_measure_peaks(ctypes.c_void_p(stream.cuda_stream), ctypes.byref(out)))
    return {"fp64_fma_tflops": out.fp64_fma_tflops, "fp32_fma_tflops": out.fp32_fma_tflops,
            "hbm_copy_gbs": out.hbm_copy_gbs, "l1_load_tbs": out.l1_load_tbs,
            "l1_load_2row_tbs": out.l1_load_2row_tbs, "lds_read_tbs": out.lds_read_tbs}


def _wrap(ptr: int, n: int) -> torch.Tensor:
    """A float64 torch view of n doubles of library-owned device memory."""
    # torch has no public from-pointer constructor for device memory; go via
    # the CUDA array interface.
    class _Holder:
        __cuda_array_interface__ = {"shape": (n,), "typestr": "<f8", "data": (ptr, False), "version": 2}
    return torch.as_tensor(_Holder(), device="cuda")
