"""FP64 CPU oracle for the SU(2) pf-FRG flow (arXiv:2109.13317).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package; the GPU library and its
Python binding never do.  It shares no code with the GPU path.

Contents
  ``pffrg_oracle.c``   plain C right-hand side and correlations on the
                       unreduced (translation-only) lattice, see its header;
  ``sites.py``         the unreduced lattice: every site within the
                       bond-distance range of each basis site (Sec. 4.1);
  ``literal.py``       a second, independent evaluation of the explicit
                       spin-index flow equations with 2x2 spin tensors and
                       complex propagators, for tiny grids;
  this module          the ctypes binding, initial conditions and the
                       explicit ODE steppers (Euler, classical RK4,
                       Dormand-Prince 5(4)).

Parity status of each function is recorded in the design notes; the pins
live in ``tests/test_oracle_*.py``.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess
import time

import numpy as np

from .sites import UnreducedLattice

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pffrg_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")


# gcc flags of the oracle: FP64 throughout, no contraction into fused
# multiply-adds and no reassociation, so the optimisation level changes no
# result bit (tests/test_oracle_sanitized.py compares an -O1 build with this one).
CFLAGS = ["-O3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC", "-shared"]


def build(force: bool = True, out: str | None = None, extra=()) -> str:
    """Compile the C oracle with gcc (FP64, no contraction, no fast-math).
    out/extra: another output path and flags (the sanitizer build of the tests)."""
    lib = out or _LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", *CFLAGS, *extra, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, lib)
    return lib


class _Lat(ctypes.Structure):
    _fields_ = [("nf", ctypes.c_int), ("w", ctypes.c_void_p), ("nb", ctypes.c_int),
                ("ns", ctypes.c_int), ("nsites", ctypes.c_void_p), ("cell", ctypes.c_void_p),
                ("bas", ctypes.c_void_p), ("rm", ctypes.c_int), ("lookup", ctypes.c_void_p),
                ("nc", ctypes.c_int)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("PFFRG_ORACLE_LIB", _LIB)
        if path == _LIB and not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        D = ctypes.c_double
        I = ctypes.c_int
        lib.orc_state_size.restype = ctypes.c_long
        lib.orc_state_size.argtypes = [P]
        lib.orc_sigma_rhs.argtypes = [P, D, P, P]
        lib.orc_sigma_rhs.restype = None
        lib.orc_rhs.argtypes = [P, D, P, P, I]
        lib.orc_rhs.restype = None
        lib.orc_vertex_rhs_element.argtypes = [P, D, P, P, I, I, I, I, I, P]
        lib.orc_vertex_rhs_element.restype = None
        lib.orc_vertex_rhs_triples.argtypes = [P, D, P, P, I, P, P, P, P, I]
        lib.orc_vertex_rhs_triples.restype = None
        lib.orc_chi.argtypes = [P, D, P, P, P]
        lib.orc_chi.restype = None
        lib.orc_chi_comps.argtypes = [P, D, P, P]
        lib.orc_chi_comps.restype = None
        lib.orc_chi_tri.argtypes = [P, D, P, P, P]
        lib.orc_chi_tri.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


class Oracle:
    """The oracle on one lattice model and one frequency mesh.

    State layout (oracle-private): sig[nf] | strain 0 | strain 1 [| 2 | 3],
    each strain [nb][n_su][nf][ns], where n_su enumerates mesh index pairs
    a >= c of (s, u) as a(a+1)/2 + c and ns pads every basis site's site
    list to the same length.  Heisenberg models (SU(2)) have two strains,
    spin and density; XYZ models (couplings (Jx, Jy, Jz), Sec. 2) four: x, y,
    z and density; general models (3x3 coupling matrices, Sec. 2) sixteen,
    Gamma^{mu nu} at index 4 mu + nu (0 the density index, 1..3 x, y, z),
    each held as r with Gamma = r where xi(mu) xi(nu) = 1 and Gamma = i r
    where it is -1 (Eq. 18).
    """

    def __init__(self, model, lattice_range: int, mesh: np.ndarray, threads: int = 0):
        self.lat = UnreducedLattice(model, lattice_range)
        self.mesh = np.ascontiguousarray(mesh, dtype=np.float64)
        self.nf = len(self.mesh)
        self.threads = int(threads)
        self.symmetry = {2: "su2", 3: "xyz", 4: "tri"}[self.lat.coupling.ndim]
        self.nc = {"su2": 2, "xyz": 4, "tri": 16}[self.symmetry]
        lat = self.lat
        self._keep = [self.mesh, lat.nsites, lat.cell, lat.bas, lat.lookup]
        self._s = _Lat(self.nf, self.mesh.ctypes.data, lat.nb, lat.ns, lat.nsites.ctypes.data,
                       lat.cell.ctypes.data, lat.bas.ctypes.data, lat.rm, lat.lookup.ctypes.data, self.nc)
        self._p = ctypes.byref(self._s)
        self.lib = _load()
        self.n_su = self.nf * (self.nf + 1) // 2
        self.size = int(self.lib.orc_state_size(self._p))
        self.vsize = lat.nb * self.n_su * self.nf * lat.ns

    # ---------------------------------------------------------- layout --
    def split(self, x: np.ndarray):
        """Views (sig, strain 0, strain 1, ...), each strain [nb, n_su, nf, ns]:
        SU(2) (sig, Gs, Gd), XYZ (sig, Gx, Gy, Gz, Gd)."""
        lat = self.lat
        sig = x[: self.nf]
        return (sig,) + tuple(x[self.nf + c * self.vsize: self.nf + (c + 1) * self.vsize]
                              .reshape(lat.nb, self.n_su, self.nf, lat.ns) for c in range(self.nc))

    def initial_state(self) -> np.ndarray:
        """Sigma = 0, spin vertices = J_ij/4 (SU(2): the spin strain; XYZ: each
        of Gx, Gy, Gz from its own coupling), density vertex = 0 (Eq. 14,
        Eq. 21)."""
        x = np.zeros(self.size)
        parts = self.split(x)
        if self.nc == 2:
            parts[1][...] = (self.lat.coupling / 4.0)[:, None, None, :]
        elif self.nc == 16:      # Gamma^{mu nu} = J^{mu nu}/4 for mu, nu = x, y, z (Eq. 22)
            for m in range(1, 4):
                for n in range(1, 4):
                    parts[1 + 4 * m + n][...] = (self.lat.coupling[:, :, m - 1, n - 1] / 4.0)[:, None, None, :]
        else:
            for c in range(3):
                parts[1 + c][...] = (self.lat.coupling[:, :, c] / 4.0)[:, None, None, :]
        return x

    # ------------------------------------------------------------- RHS --
    def sigma_rhs(self, lam: float, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.zeros(self.nf)
        self.lib.orc_sigma_rhs(self._p, float(lam), _ptr(x), _ptr(out))
        return out

    def rhs(self, lam: float, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.zeros(self.size)
        self.lib.orc_rhs(self._p, float(lam), _ptr(x), _ptr(out), self.threads)
        return out

    def vertex_rhs_element(self, lam, x, dsig, b, k, a, t, c):
        x = np.ascontiguousarray(x, dtype=np.float64)
        dsig = np.ascontiguousarray(dsig, dtype=np.float64)
        out = np.zeros(self.nc)
        self.lib.orc_vertex_rhs_element(self._p, float(lam), _ptr(x), _ptr(dsig),
                                        int(b), int(k), int(a), int(t), int(c), _ptr(out))
        return out

    def vertex_rhs_triples(self, lam, x, dsig, triples) -> np.ndarray:
        """Flow of every (basis, site) element at each (a, t, c) triple:
        returns [nq, nb, ns, strains]."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        dsig = np.ascontiguousarray(dsig, dtype=np.float64)
        tr = np.asarray(triples, dtype=np.int32).reshape(-1, 3)
        a = np.ascontiguousarray(tr[:, 0]); t = np.ascontiguousarray(tr[:, 1])
        c = np.ascontiguousarray(tr[:, 2])
        out = np.zeros((len(tr), self.lat.nb, self.lat.ns, self.nc))
        self.lib.orc_vertex_rhs_triples(self._p, float(lam), _ptr(x), _ptr(dsig), len(tr),
                                        _ptr(a), _ptr(t), _ptr(c), _ptr(out), self.threads)
        return out

    def chi_comps(self, lam: float, x: np.ndarray) -> np.ndarray:
        """chi per strain, [strains, nb, ns] (SU(2): zz, 00; XYZ: xx, yy, zz, 00)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.zeros((self.nc, self.lat.nb, self.lat.ns))
        self.lib.orc_chi_comps(self._p, float(lam), _ptr(x), _ptr(out))
        return out

    def chi_tri(self, lam: float, x: np.ndarray):
        """TRI: chi^{mu nu} for mu, nu = 0..3, real and imaginary parts, each
        [4, 4, nb, ns] (Eq. 30 from the spin tensors)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        re = np.zeros((4, 4, self.lat.nb, self.lat.ns))
        im = np.zeros((4, 4, self.lat.nb, self.lat.ns))
        self.lib.orc_chi_tri(self._p, float(lam), _ptr(x), _ptr(re), _ptr(im))
        return re, im

    def chi_k_xyz(self, chi: np.ndarray, kpts: np.ndarray) -> np.ndarray:
        """XYZ structure factor (Eq. 31) per unit cell:
        (1/nb) sum_b sum_{j in range of b} cos(k.(r_b - r_j)) (chi^xx + chi^yy + chi^zz)_bj."""
        kpts = np.asarray(kpts, dtype=np.float64).reshape(-1, 3)
        out = np.zeros(len(kpts))
        lat = self.lat
        for b in range(lat.nb):
            n = lat.nsites[b]
            dr = lat.basis_pos[b][None, :] - lat.site_pos[b, :n]
            out += np.cos(kpts @ dr.T) @ (chi[0, b, :n] + chi[1, b, :n] + chi[2, b, :n])
        return out / lat.nb

    def chi(self, lam: float, x: np.ndarray):
        """SU(2): (chi_zz, chi_dd), each [nb, ns] over the unreduced site lists."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        zz = np.zeros((self.lat.nb, self.lat.ns))
        dd = np.zeros((self.lat.nb, self.lat.ns))
        self.lib.orc_chi(self._p, float(lam), _ptr(x), _ptr(zz), _ptr(dd))
        return zz, dd

    def chi_k(self, chi_zz: np.ndarray, kpts: np.ndarray) -> np.ndarray:
        """Structure factor (Eq. 31) per unit cell:
        (1/nb) sum_b sum_{j in range of b} cos(k.(r_b - r_j)) 3 chi^zz_bj."""
        kpts = np.asarray(kpts, dtype=np.float64).reshape(-1, 3)
        out = np.zeros(len(kpts))
        lat = self.lat
        for b in range(lat.nb):
            n = lat.nsites[b]
            dr = lat.basis_pos[b][None, :] - lat.site_pos[b, :n]
            phase = kpts @ dr.T
            out += np.cos(phase) @ (3.0 * chi_zz[b, :n])
        return out / lat.nb

    # ----------------------------------------------------------- flows --
    def euler_step(self, lam0, lam1, x):
        """One Euler step (Eq. 42): x(lam1) = x(lam0) + (lam1 - lam0) dx/dlam."""
        return x + (lam1 - lam0) * self.rhs(lam0, x)

    def rk4_step(self, lam0, lam1, x):
        """Classical fourth-order Runge-Kutta step in Lambda from lam0 to lam1."""
        h = lam1 - lam0
        lm = lam0 + 0.5 * h
        k1 = self.rhs(lam0, x)
        k2 = self.rhs(lm, x + (0.5 * h) * k1)
        k3 = self.rhs(lm, x + (0.5 * h) * k2)
        k4 = self.rhs(lam1, x + h * k3)
        return x + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)

    def dopri_flow(self, lam_start, lam_stop, rtol, atol, h0, hmin, x0=None, max_steps=0,
                   observer=None):
        """Adaptive Dormand-Prince 5(4) flow of this model from lam_start down
        to lam_stop (see ``dopri_integrate``).  The right-hand side jumps where
        Lambda crosses w_n/2 (a step function of a delta-point propagator
        switches, Eq. 12), so those cutoffs are the breakpoints.
        Returns (x, accepted cutoffs)."""
        x = self.initial_state() if x0 is None else np.array(x0, dtype=np.float64)
        return dopri_integrate(self.rhs, x, lam_start, lam_stop, rtol, atol, h0, hmin,
                               breakpoints=[0.5 * w for w in self.mesh], max_steps=max_steps,
                               observer=observer)

    def flow(self, schedule, x0=None, scheme="rk4", observer=None):
        """Integrate along a fixed cutoff schedule; observer(lam, x) after each step."""
        x = self.initial_state() if x0 is None else np.array(x0, dtype=np.float64)
        step = {"rk4": self.rk4_step, "euler": self.euler_step}[scheme]
        for i in range(len(schedule) - 1):
            x = step(float(schedule[i]), float(schedule[i + 1]), x)
            if observer is not None:
                observer(float(schedule[i + 1]), x)
        return x



# ---------------------------------------------------------------------------
# Dormand-Prince 5(4) (J. R. Dormand and P. J. Prince, "A family of embedded
# Runge-Kutta formulae", J. Comput. Appl. Math. 6 (1980) 19-26): nodes, stage
# coefficients, and the difference of the 5th and 4th order weights.  The
# seventh stage is evaluated at the accepted 5th-order point, so it serves as
# the first stage of the next step.
DP_C = (0.0, 1 / 5, 3 / 10, 4 / 5, 8 / 9, 1.0, 1.0)
DP_A = ((), (1 / 5,), (3 / 40, 9 / 40), (44 / 45, -56 / 15, 32 / 9),
        (19372 / 6561, -25360 / 2187, 64448 / 6561, -212 / 729),
        (9017 / 3168, -355 / 33, 46732 / 5247, 49 / 176, -5103 / 18656),
        (35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84))
DP_E = (35 / 384 - 5179 / 57600, 0.0, 500 / 1113 - 7571 / 16695, 125 / 192 - 393 / 640,
        -2187 / 6784 + 92097 / 339200, 11 / 84 - 187 / 2100, -1 / 40)


def dopri_step(rhs, l, dl, x, k0):
    """One Dormand-Prince 5(4) step in l = ln Lambda of dx/dl = Lambda dx/dLambda
    (rhs(Lambda, x) = dx/dLambda) from l to l + dl, with k0 = rhs(exp(l), x).
    Returns (y, e, k): the 5th-order point, the difference of the 5th- and
    4th-order points, and the seven stage derivatives dx/dLambda."""
    lam = [math.exp(l + c * dl) for c in DP_C]
    k = [k0] + [None] * 6
    y = x
    for i in range(1, 7):
        y = x.copy()
        for j in range(i):
            cj = dl * DP_A[i][j] * lam[j]
            if cj != 0.0:
                y += cj * k[j]
        k[i] = rhs(lam[i], y)
    e = np.zeros_like(x)
    for j in range(7):
        cj = dl * DP_E[j] * lam[j]
        if cj != 0.0:
            e += cj * k[j]
    return y, e, k


def dopri_integrate(rhs, x0, lam_start, lam_stop, rtol, atol, h0, hmin, breakpoints=(),
                    max_steps=0, observer=None):
    """Adaptive Dormand-Prince 5(4) in l = ln Lambda from lam_start down to
    lam_stop.  Error norm max_i |e_i| / (atol + rtol max(|x_i|, |y_i|));
    accept if <= 1.  Step sizes are h0 2^(m/4); after a step m changes by
    round(4 log2(f)) with f = clamp(0.9 err^-1/5, 0.2, 5) (rejected: clamp to
    [0.2, 1] and at least -1); a step shortened to land on a breakpoint or the
    end keeps m unless f < 1.  Across a breakpoint of the right-hand side (a
    cutoff where it jumps) a step ends 1e-12 (in l) above it and the next one
    starts 1e-12 below it, with the derivative evaluated afresh.
    observer(Lambda, x) after each accepted step.  Returns (x, accepted
    cutoffs)."""
    x = np.array(x0, dtype=np.float64)
    lend = math.log(lam_stop)
    l = math.log(lam_start)
    m = 0

    def ladder(mm):
        return h0 * 2.0 ** (mm / 4.0)

    def quarter_steps(f):
        v = 4.0 * math.log2(f)
        return int(math.floor(v + 0.5)) if v >= 0 else -int(math.floor(-v + 0.5))

    maxs = max_steps if max_steps > 0 else 1000000
    brk = sorted((math.log(b) for b in breakpoints if lend < math.log(b) < l), reverse=True)
    gap = 1e-12
    ib = 0
    k0 = rhs(math.exp(l), x)
    lams = []
    attempts = 0
    while l > lend:
        attempts += 1
        if attempts > 50 * maxs:
            raise RuntimeError("too many rejected steps")
        while ib < len(brk) and brk[ib] + gap >= l:
            ib += 1
        dl = -ladder(m)
        last = at_brk = False
        if ib < len(brk) and l + dl <= brk[ib] + gap:
            dl = (brk[ib] + gap) - l
            at_brk = True
        if l + dl <= lend:
            dl = lend - l
            last, at_brk = True, False
        y, e, k = dopri_step(rhs, l, dl, x, k0)
        fin = bool(np.all(np.isfinite(y)) and np.all(np.isfinite(x)))
        err = float(np.max(np.abs(e) / (atol + rtol * np.maximum(np.abs(x), np.abs(y))))) if fin else 0.0
        if fin and err <= 1.0:
            x = y
            k0 = k[6]
            l = lend if last else l + dl
            if at_brk:
                l = brk[ib] - gap
                ib += 1
                k0 = rhs(math.exp(l), x)
            lams.append(math.exp(l))
            if observer is not None:
                observer(math.exp(l), x)
            if len(lams) >= maxs:
                break
            fac = min(5.0, max(0.2, 0.9 * err ** -0.2)) if err > 0.0 else 5.0
            dm = quarter_steps(fac)
            if not (at_brk or last) or dm < 0:
                m += dm
        else:
            fac = min(1.0, max(0.2, 0.9 * err ** -0.2)) if (fin and err > 0.0) else 0.2
            m += min(-1, quarter_steps(fac))
        if ladder(m) < hmin and l > lend:
            raise RuntimeError(f"adaptive step fell below hmin at lambda = {math.exp(l)}")
    return x, lams

def timed(fn, *a, **kw):
    t0 = time.perf_counter()
    r = fn(*a, **kw)
    return r, time.perf_counter() - t0
