"""Literal spin-index evaluation of the pf-FRG flow equations, tiny grids only.

TEST INFRASTRUCTURE ONLY.  An independent second evaluation of what the C
oracle computes, written straight from the paper's explicit equations:

  * the vertex is built as 16 basis functions Gamma^{mu nu} (Eq. 16) with the
    SU(2) constraint (Gamma^{11}=Gamma^{22}=Gamma^{33}, off-diagonals zero),
    for XYZ states the XYZ constraint (the four diagonal components
    Gamma^{00}, Gamma^{11}, Gamma^{22}, Gamma^{33} free, off-diagonals zero),
    and for general (TRI) states all sixteen, complex where Eq. 18 makes
    them imaginary;
    values outside the stored octant come from the general symmetry relations
    (Eq. 18, with xi of Eq. 19 and mu<->nu transposition applied literally);
  * the spin tensor Gamma^{a'b';ab} = Gamma^{mu nu} sigma^mu_{a'a} sigma^nu_{b'b}
    (Eq. 25) enters the explicit flow equations (Eq. 23, Eq. 24) with every
    spin sum done numerically;
  * propagators are complex: G = theta(|w|-L)/(iw - Sigma), S with its delta
    function (Eq. 12), Skat = S - G^2 dSigma/dLambda (Eq. 13);
  * the results are projected back on Gamma^{mu nu} by Pauli traces, so the
    SU(2) closure (off-diagonal and 11/22/33 components) can be checked.

Quadrature readings are the same as the C oracle's (delta parts analytic at
|w| = Lambda, trapezoid on mesh points inside the Katanin domain), but the
node set is built by a different procedure (filter + sort of candidates).
"""

from __future__ import annotations

import numpy as np

SIG = np.array([[[1, 0], [0, 1]],
                [[0, 1], [1, 0]],
                [[0, -1j], [1j, 0]],
                [[1, 0], [0, -1]]], dtype=np.complex128)
XI = np.array([1.0, -1.0, -1.0, -1.0])
XIXI = np.outer(XI, XI)


class LiteralFlow:
    """Evaluate the flow on an oracle state (layout of ``oracle.Oracle``)."""

    def __init__(self, orc):
        self.o = orc
        self.lat = orc.lat
        self.w = orc.mesh
        self.nf = orc.nf
        self.wmax = float(self.w[-1])

    # ------------------------------------------------------ look-ups --
    def _bracket(self, x):
        w = self.w
        if x <= w[0]:
            return (0, 0), (1.0, 0.0)
        if x >= w[-1]:
            return (self.nf - 1, self.nf - 1), (1.0, 0.0)
        i = int(np.searchsorted(w, x, side="right")) - 1
        h = w[i + 1] - w[i]
        return (i, i + 1), ((w[i + 1] - x) / h, (x - w[i]) / h)

    def _stored(self, b, k, a, t, c):
        """Gamma^{mu nu} at mesh indices; corners with s < u via the s<->u relation."""
        if a < c:
            m = self._stored(b, k, c, t, a)
            return m * (-XI)[None, :]
        su = a * (a + 1) // 2 + c
        parts = self.o.split(self.x)
        if self.o.nc == 16:
            # general state: Gamma^{mu nu} = r or i r by xi(mu) xi(nu) (Eq. 18)
            r = np.array([parts[1 + q][b, su, t, k] for q in range(16)]).reshape(4, 4)
            return np.where(XIXI > 0, 1.0, 1j) * r
        m = np.zeros((4, 4))
        if self.o.nc == 2:
            _, gs, gd = parts
            m[0, 0] = gd[b, su, t, k]
            m[1, 1] = m[2, 2] = m[3, 3] = gs[b, su, t, k]
        else:
            _, gx, gy, gz, gd = parts
            m[0, 0] = gd[b, su, t, k]
            m[1, 1], m[2, 2], m[3, 3] = gx[b, su, t, k], gy[b, su, t, k], gz[b, su, t, k]
        return m

    def gamma(self, b1, d, b2, s, t, u):
        """4x4 matrix Gamma^{mu nu}_{i1 i2}(s,t,u), i1 = (cell 0, b1), i2 = (cell d, b2)."""
        d = tuple(int(v) for v in d)
        if s < 0:   # Gamma^{mu nu}_{i1i2}(s,t,u) = Gamma^{nu mu}_{i2i1}(-s,t,u)
            return self.gamma(b2, tuple(-v for v in d), b1, -s, t, u).T
        if t < 0:   # = xi(mu) xi(nu) Gamma^{mu nu}(s,-t,u)
            return XIXI * self.gamma(b1, d, b2, s, -t, u)
        if u < 0:   # = xi(mu) xi(nu) Gamma^{nu mu}_{i2i1}(s,t,-u)
            return XIXI * self.gamma(b2, tuple(-v for v in d), b1, s, t, -u).T
        if s < u:   # = -xi(nu) Gamma^{mu nu}(u,t,s)
            return self.gamma(b1, d, b2, u, t, s) * (-XI)[None, :]
        k = self.lat.index(b1, d, b2)
        if k < 0:
            return np.zeros((4, 4), dtype=np.complex128)
        (sa, sb), (fs0, fs1) = self._bracket(s)
        (ta, tb), (ft0, ft1) = self._bracket(t)
        (ua, ub), (fu0, fu1) = self._bracket(u)
        acc = np.zeros((4, 4), dtype=np.complex128)
        for ui, fu in ((ua, fu0), (ub, fu1)):
            for ti, ft in ((ta, ft0), (tb, ft1)):
                for si, fs in ((sa, fs0), (sb, fs1)):
                    wgt = fu * ft * fs
                    if wgt != 0.0:
                        acc += wgt * self._stored(b1, k, si, ti, ui)
        return acc

    def spin_tensor(self, b1, d, b2, s, t, u):
        """V[a', b', a, b] = Gamma^{mu nu} sigma^mu_{a'a} sigma^nu_{b'b} (Eq. 25)."""
        g = self.gamma(b1, d, b2, s, t, u)
        return np.einsum("mn,mpa,nqb->pqab", g, SIG, SIG)

    # ---------------------------------------------------- propagators --
    def _odd(self, v, x):
        sg = 1.0
        if x < 0:
            x, sg = -x, -1.0
        (i0, i1), (f0, f1) = self._bracket(x)
        return sg * (f0 * v[i0] + f1 * v[i1])

    def Sigma(self, x):
        return 1j * self._odd(self.x[: self.nf], x)

    def dSigma(self, x):
        return 1j * self._odd(self.dsig, x)

    def G(self, x, tie=1.0):
        a = abs(x)
        th = 1.0 if a > self.lam else (tie if a == self.lam else 0.0)
        if th == 0.0:
            return 0.0
        return th / (1j * x - self.Sigma(x))

    def G_in(self, x):
        """G at a quadrature node of the Katanin domain: the step function is 1
        on the closed domain, also where rounding puts |x| a hair below Lambda
        at a domain edge."""
        return 1.0 / (1j * x - self.Sigma(x))

    def Sfac(self, x):
        """Residue of S at its delta point: 1/(ix - Sigma(x))."""
        return 1.0 / (1j * x - self.Sigma(x))

    # ------------------------------------------------------ self-energy --
    def sigma_rhs(self, lam, x):
        """dSigma/dLambda (Eq. 23), returned as the imaginary part sig'."""
        self.lam, self.x = float(lam), x
        out = np.zeros(self.nf, dtype=np.complex128)
        lat = self.lat
        for n, w1 in enumerate(self.w):
            acc = 0.0j
            for x2 in (lam, -lam):
                val = 0.0j
                for a2 in range(2):
                    for k in range(lat.nsites[0]):
                        V = self.spin_tensor(0, lat.cell[0, k], lat.bas[0, k], w1 + x2, 0.0, w1 - x2)
                        val += V[0, a2, 0, a2]
                    V0 = self.spin_tensor(0, (0, 0, 0), 0, w1 + x2, x2 - w1, 0.0)
                    val -= V0[a2, 0, 0, a2]
                acc += val * self.Sfac(x2)
            out[n] = -acc / (2.0 * np.pi)
        return out

    # ------------------------------------------------------ quadrature --
    def nodes(self, partner=None):
        """Trapezoid nodes/weights on {|w|>=L, |partner(w)|>=L} within [-wmax, wmax]
        (without a partner: on {|w|>=L} within [-wmax, wmax])."""
        lam, wmax = self.lam, self.wmax
        cands = list(self.w) + list(-self.w) + [lam, -lam, wmax, -wmax]
        if partner is not None:
            p0, p1 = partner(0.0), partner(1.0)
            c = -p0 / (p1 - p0)          # zero of the partner argument
            cands += [c - lam, c + lam]

        def inside(v):
            # D is [-wmax, wmax] minus the open intervals where |w| < lam or
            # |partner(w)| < lam; membership is decided against the interval
            # ends c -+ lam so that the ends themselves belong to D exactly.
            if partner is not None and c - lam < v < c + lam:
                return False
            return not (-lam < v < lam) and -wmax <= v <= wmax

        pts = sorted(set(v for v in cands if inside(v)))
        wts = np.zeros(len(pts))
        for i in range(len(pts) - 1):
            mid = 0.5 * (pts[i] + pts[i + 1])
            if inside(mid):
                hseg = pts[i + 1] - pts[i]
                wts[i] += 0.5 * hseg
                wts[i + 1] += 0.5 * hseg
        return pts, wts

    def bubble_integral(self, partner, pinv, F):
        """(1/2pi) int dw [G(w) Skat(p(w)) + G(p(w)) Skat(w)] F(w)."""
        lam = self.lam
        acc = 0.0
        for xx in (lam, -lam):
            acc = acc + self.G(pinv(xx), tie=0.5) * self.Sfac(xx) * F(pinv(xx))
            acc = acc + self.G(partner(xx), tie=0.5) * self.Sfac(xx) * F(xx)
        pts, wts = self.nodes(partner)
        for w, wt in zip(pts, wts):
            if wt == 0.0:
                continue
            p = partner(w)
            kat = self.G_in(w) * (-self.G_in(p) ** 2 * self.dSigma(p)) + self.G_in(p) * (-self.G_in(w) ** 2 * self.dSigma(w))
            acc = acc + wt * kat * F(w)
        return acc / (2.0 * np.pi)

    # ---------------------------------------------------- vertex flow --
    def vertex_rhs(self, lam, x, dsig, b, k, a, it, c):
        """Gamma^{mu nu} flow (4x4, complex) of one stored element, Eq. 24."""
        lat = self.lat
        return self.vertex_rhs_at(lam, x, dsig, b, tuple(lat.cell[b, k]), int(lat.bas[b, k]),
                                  self.w[a], self.w[it], self.w[c])

    def vertex_rhs_at(self, lam, x, dsig, b, dk, bk, s, t, u):
        """Gamma^{mu nu}_{i1 i2} flow at arbitrary transfer frequencies (s,t,u),
        i1 = (cell 0, b), i2 = (cell dk, bk)."""
        self.lam, self.x, self.dsig = float(lam), x, dsig
        lat = self.lat
        w1p, w2p = 0.5 * (s + t + u), 0.5 * (s - t - u)
        w1, w2 = 0.5 * (s - t + u), 0.5 * (s + t - u)
        dk = tuple(int(v) for v in dk); bk = int(bk)
        zero = (0, 0, 0)

        def V(b1, d, b2, S, T, U):
            return self.spin_tensor(b1, d, b2, S, T, U)

        def Fs(w):
            A = V(b, dk, bk, s, w1p - w, w - w2p)          # legs (1',2';3,4)
            B = V(b, dk, bk, s, w - w1, w - w2)            # legs (3,4;1,2)
            return np.einsum("pqcd,cdab->pqab", A, B)

        def Ft(w):
            tot = np.zeros((2, 2, 2, 2), dtype=np.complex128)
            for j in range(lat.nsites[b]):
                dj = tuple(lat.cell[b, j]); bj = int(lat.bas[b, j])
                d2 = tuple(dk[i] - dj[i] for i in range(3))
                if lat.index(bj, d2, bk) < 0:
                    continue
                A = V(b, dj, bj, w1 + w, t, w1p - w)       # legs (1',4;1,3)
                B = V(bj, d2, bk, w + w2p, t, w - w2)      # legs (3,2';4,2)
                tot -= np.einsum("pdac,cqdb->pqab", A, B)
            A = V(b, dk, bk, w1 + w, t, w1p - w)           # legs (1',4;1,3)
            O1 = V(bk, zero, bk, w2p + w, w2 - w, -t)      # legs (2',3;4,2)
            tot += np.einsum("pdac,qcdb->pqab", A, O1)
            O2 = V(b, zero, b, w1 + w, w - w1p, -t)        # legs (4,1';1,3)
            B = V(b, dk, bk, w + w2p, t, w - w2)           # legs (3,2';4,2)
            tot += np.einsum("dpac,cqdb->pqab", O2, B)
            return tot

        def Fu(w):
            A = V(b, dk, bk, w1 + w, w - w2p, u)           # legs (4,2';1,3)
            B = V(b, dk, bk, w1p + w, w2 - w, u)           # legs (1',3;4,2)
            return np.einsum("dqac,pcdb->pqab", A, B)

        tot = self.bubble_integral(lambda w: s - w, lambda y: s - y, Fs)
        tot = tot + self.bubble_integral(lambda w: w - t, lambda y: y + t, Ft)
        tot = tot + self.bubble_integral(lambda w: u + w, lambda y: y - u, Fu)
        # project on the basis functions: Gamma^{mu nu} = 1/4 sum V sigma^mu_{a a'} sigma^nu_{b b'}
        return 0.25 * np.einsum("pqab,map,nbq->mn", tot, SIG, SIG)

    # ---------------------------------------------------- correlations --
    def chi(self, lam, x, b, k, mu):
        """chi^{mu mu}_{ij} from Eq. 30 (one-loop term with delta_ij)."""
        self.lam, self.x = float(lam), x
        lat = self.lat
        pts, wts = self.nodes()
        dk = tuple(lat.cell[b, k]); bk = int(lat.bas[b, k])
        sm = SIG[mu]
        acc = 0.0j
        if k == 0:
            for w, wt in zip(pts, wts):
                acc += -1.0 / (8.0 * np.pi) * wt * self.G(w) ** 2 * np.trace(sm @ sm)
        for w1, a1 in zip(pts, wts):
            for w2, a2 in zip(pts, wts):
                # Gamma((i,w1,a1'),(j,w2,a2');(i,w1,a1),(j,w2,a2)) incl. -(1'<->2')
                Vd = self.spin_tensor(b, dk, bk, w1 + w2, 0.0, w1 - w2)     # [a1',a2',a1,a2]
                full = Vd.copy()
                if k == 0:
                    Ve = self.spin_tensor(b, (0, 0, 0), b, w1 + w2, w2 - w1, 0.0)  # legs (2',1';1,2)
                    full = full - np.einsum("qpab->pqab", Ve)
                val = np.einsum("ap,bq,pqab->", sm, sm, full)
                acc += -1.0 / (16.0 * np.pi ** 2) * a1 * a2 * self.G(w1) ** 2 * self.G(w2) ** 2 * val
        return acc
