"""Emitter importance sampling combined with cosine sampling by multiple
importance sampling (next-event estimation on emissive surfels) for the path
tracer of Sec. 3.4 (Eq. 9), float64.

The paper proposes this as the remedy for the noise of small emitters
(Sec. 5, limitations; Appendix D, Discussion) without fixing an estimator.
The reading built here:

* Emitters: the surfels with e > tau_E and opacity > 0. A segment's
  composited E is a sum of the e of its hits with weights that add up to
  A <= 1, so a segment passes the emitter test (Eq. 5) only if it blends one
  of these surfels (with tau_E >= 0).
* Selection: emitter j with probability w_j / W, w_j = sigma_j s_u s_v
  (rbar_j + e_j), rbar the mean of r's three channels, W = sum_j w_j; by
  inversion on u0: the first j whose inclusive prefix sum exceeds u0 W.
* Point: uniform on the j's k_sigma ellipse, y = p + k sqrt(u1) (s_u cos(2 pi
  u2) t_u + s_v sin(2 pi u2) t_v). Its area density on that ellipse is
  rho_j = (w_j / W) / (pi k^2 s_u s_v) = sigma_j (rbar_j + e_j) / (pi k^2 W).
* Light segment: from the vertex X along w_l = (y - X) / |y - X|, traced like
  any other segment (every surfel on the ray is blended); its emitter part is
  R if E > tau_E, else 0.
* Light pdf in solid angle: p_l(X, w) = sum over the emitters j whose ellipse
  the ray X + d w crosses at d > 0 (|w.n_j| > 1e-12 and u^2 + v^2 <= k^2, the
  tracer's acceptance test without t_min) of rho_j d^2 / |w.n_j|.
* Cosine pdf about the vertex normal: p_b(w) = max(0, w.Nt) / pi.
* Power heuristic, exponent 2. With beta the throughput after the vertex's
  P (before Russian roulette), a light segment with w_l.Nt > 0 adds
  beta R p_b p_l / (p_b^2 + p_l^2) (that is f cos / p_l times the light weight
  p_l^2 / (p_b^2 + p_l^2), f = P / pi); a cosine-sampled segment k >= 1 that
  passes the emitter test adds beta R p_b^2 / (p_b^2 + p_l^2) and ends the
  path. The camera segment (k = 0) is not weighted. Everything else (depth
  limit, Russian roulette, the sample stream of the cosine direction) is the
  plain path tracer's.
* Sample stream: the light sample at the vertex after segment k uses the
  Philox counter (pixel, sample, 2^31 + k, id); u0 selects, u1 and u2 place
  the point.
* Selection by cells (an option, cell size c > 0, a power of two): the
  emitters are grouped by the cube of side c holding their centre, in the
  order (cell, surfel index); at the vertex X, a cell is chosen with
  probability I_c / sum I over the cells, I_c = W_c / max(|X - m_c|^2, c^2)
  (W_c the cell's summed w, m_c its centre), by inversion on u0, and an
  emitter of the cell with probability w_j / W_c by inversion on u3 (the
  counter's fourth word). The area density of emitter j becomes
  (I_c(X) / sum I) sigma_j (rbar_j + e_j) / (pi k^2 W_c): emitters near the
  vertex are drawn more often, and those of other rooms seldom.

The two weights add up to one wherever one of the strategies can produce a
direction, and p_l > 0 wherever the emitter part is not zero, so the
estimator has the expectation of the plain path tracer's, with less variance
where emitters are small.

Decision margins: besides the tracer's own flags, F_NEE marks a path where
another rounding of the same definition may select another emitter (u0 W
within the prefix sums' rounding of a boundary), flip the sign test of
w_l.Nt, or count another crossing in p_l (u^2 + v^2 near k^2, d near 0).

Pinned by tests/test_oracle_nee.py: p_l integrates to one over the sphere
(uniform-sphere Monte Carlo), the mean of 1 / p_l over light samples is the
solid angle the emitters cover (counted by uniform directions), the
selection frequencies w_j / W (and, with cells, I_c / sum I times w_j / W_c)
and the uniform point density on the ellipse, for both selections,
the single-bounce integral of one emitter over one receiver by quadrature
(scipy dblquad), equal means of this estimator and the plain path tracer on a
room, and per-sample equality with the plain path tracer when no vertex is
reached (max_depth 0).
"""
import numpy as np

from . import philox
from .frames import cosine_direction
from .render import _camera, _pixels
from .tracer import KAPPA, UGEOM, F_RR, UF32, Scene64, trace

NEE_SEGMENT = 1 << 31
F_NEE = 1 << 9


class Emitters:
    """The emitter table of a scene for a threshold tau_E.

    cell = 0: selection by power alone (w_j / W). cell = c > 0 (a power of
    two): emitters are grouped by the cube of side c that holds their centre
    (floor of the float32 centre / c per axis) and taken in the order (cell,
    surfel index); at a vertex X a cell is chosen with probability
    I_c / sum I, I_c = W_c / max(|X - m_c|^2, c^2), W_c the cell's summed w
    and m_c its centre, by inversion on u0 over the cells in order, then an
    emitter of the cell with probability w_j / W_c by inversion on u3."""

    def __init__(self, sc: Scene64, tau_E: float, k_sigma: float = 3.0, cell: float = 0.0):
        self.tau_E = float(tau_E)
        self.k = float(k_sigma)
        self.cell = float(cell)
        j = np.nonzero((sc.e > np.float64(np.float32(tau_E))) & (sc.sigma > 0))[0]
        if self.cell > 0 and j.size:
            ic = np.floor(sc.p[j] / self.cell)
            order = np.lexsort((j, ic[:, 2], ic[:, 1], ic[:, 0]))
            j = j[order]
        self.idx = j
        rbar = sc.r[j].sum(axis=1) / 3.0
        self.w = sc.sigma[j] * sc.su[j] * sc.sv[j] * (rbar + sc.e[j])
        self.cdf = np.cumsum(self.w)
        self.W = float(self.cdf[-1]) if j.size else 0.0
        self.p, self.tu, self.tv, self.n = sc.p[j], sc.tu[j], sc.tv[j], sc.n[j]
        self.su, self.sv = sc.su[j], sc.sv[j]
        self.pmax = np.abs(self.p).max(axis=1) if j.size else np.zeros(0)
        self.smin = np.minimum(self.su, self.sv)
        if self.cell > 0 and j.size:
            ic = np.floor(self.p / self.cell)
            first = np.ones(j.size, dtype=bool)
            first[1:] = np.any(ic[1:] != ic[:-1], axis=1)
            self.cell_of = np.cumsum(first) - 1
            self.begin = np.nonzero(first)[0]
            self.end = np.append(self.begin[1:], j.size)
            self.ctr = (ic[self.begin] + 0.5) * self.cell
            # per-cell sums and prefix sums, each summed in order within its cell
            self.cdf_in = np.zeros(j.size)
            self.Wc = np.zeros(self.begin.size)
            for c, (b, e) in enumerate(zip(self.begin, self.end)):
                self.cdf_in[b:e] = np.cumsum(self.w[b:e])
                self.Wc[c] = self.cdf_in[e - 1]
            # area density of the point sampler given the emitter's cell
            self.rho = sc.sigma[j] * (rbar + sc.e[j]) / (np.pi * self.k * self.k * self.Wc[self.cell_of])
        else:
            # area density of the point sampler on each ellipse
            self.rho = (sc.sigma[j] * (rbar + sc.e[j]) / (np.pi * self.k * self.k * self.W)) if j.size else np.zeros(0)

    def importance(self, X):
        """I_c(X) [M, cells] and their sums [M] (cell mode)."""
        X = np.atleast_2d(X)
        d = X[:, None, :] - self.ctr[None, :, :]
        d2 = d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2]
        I = self.Wc[None, :] / np.maximum(d2, self.cell * self.cell)
        return I, np.cumsum(I, axis=1)[:, -1]

    @property
    def count(self):
        return int(self.idx.size)

    def sample(self, u0, u1, u2, u3=None, X=None, eX=None):
        """Emitter (position in the table), point y [M,3] and the selection
        margin flag for uniforms u0, u1, u2 (u3) [M] at vertices X [M,3]
        (cell mode; eX their error bounds)."""
        if self.cell > 0:
            j, amb = self._select_cells(np.asarray(u0), np.asarray(u3), np.atleast_2d(X),
                                        np.zeros(len(u0)) if eX is None else np.asarray(eX))
        else:
            x = np.asarray(u0) * self.W
            j = np.searchsorted(self.cdf, x, side="right")
            j = np.minimum(j, self.count - 1)
            # the prefix sums of another summation order differ by ~count * U * W
            tol = 4.0 * self.count * 2.0 ** -53 * self.W
            lo = np.where(j > 0, self.cdf[np.maximum(j - 1, 0)], -np.inf)
            amb = (np.abs(x - self.cdf[j]) <= tol) | (np.abs(x - lo) <= tol)
        r = self.k * np.sqrt(u1)
        phi = 2.0 * np.pi * np.asarray(u2)
        a = (r * np.cos(phi) * self.su[j])[:, None]
        b = (r * np.sin(phi) * self.sv[j])[:, None]
        y = self.p[j] + a * self.tu[j] + b * self.tv[j]
        return j, y, amb

    def _select_cells(self, u0, u3, X, eX):
        I, S = self.importance(X)
        cum = np.cumsum(I, axis=1)
        x = u0 * S
        c = np.minimum((cum <= x[:, None]).sum(axis=1), self.Wc.size - 1)
        # I moves with X by about 2 |dX| / distance, and another summation
        # order by a few roundings per cell
        d2min = np.maximum(np.min(np.sum((X[:, None, :] - self.ctr[None]) ** 2, axis=2), axis=1), self.cell ** 2)
        tol = S * (4.0 * eX / np.sqrt(d2min) + 8.0 * self.Wc.size * 2.0 ** -53) + 1e-300
        rows = np.arange(X.shape[0])
        lo = np.where(c > 0, cum[rows, np.maximum(c - 1, 0)], -np.inf)
        amb = (np.abs(x - cum[rows, c]) <= tol) | (np.abs(x - lo) <= tol)
        # the emitter within the cell
        b, e = self.begin[c], self.end[c]
        y = u3 * self.Wc[c]
        j = np.empty(c.size, dtype=np.int64)
        for m in range(c.size):
            k = b[m] + np.searchsorted(self.cdf_in[b[m]:e[m]], y[m], side="right")
            j[m] = min(k, e[m] - 1)
        tin = 4.0 * (e - b) * 2.0 ** -53 * self.Wc[c]
        lo_in = np.where(j > b, self.cdf_in[np.maximum(j - 1, 0)], -np.inf)
        amb |= (np.abs(y - self.cdf_in[j]) <= tin) | (np.abs(y - lo_in) <= tin)
        return j, amb

    def pdf(self, X, W, eX=None, ew=None):
        """Solid-angle density p_l of the light sampler for rays X [M,3] + d W
        [M,3] (unit), and a margin flag per ray (eX, ew: the ray's origin and
        direction error bounds, as for the tracer)."""
        X = np.atleast_2d(X)
        W = np.atleast_2d(W)
        M = X.shape[0]
        if self.count == 0:
            return np.zeros(M), np.zeros(M, dtype=bool)
        eX = np.zeros(M) if eX is None else np.asarray(eX, dtype=np.float64)
        ew = np.zeros(M) if ew is None else np.asarray(ew, dtype=np.float64)
        k2 = self.k * self.k
        d = self.p[None, :, :] - X[:, None, :]                      # [M, E, 3]
        den = W @ self.n.T                                           # [M, E]
        num = np.einsum("mec,ec->me", d, self.n)
        valid = np.abs(den) > 1e-12
        with np.errstate(divide="ignore", invalid="ignore"):
            t = np.where(valid, num / np.where(valid, den, 1.0), np.inf)
        y = np.where(valid[..., None], t[..., None] * W[:, None, :] - d, 0.0)
        u = np.einsum("mec,ec->me", y, self.tu) / self.su[None]
        v = np.einsum("mec,ec->me", y, self.tv) / self.sv[None]
        q2 = u * u + v * v
        cross = valid & (t > 0.0) & (q2 <= k2)
        with np.errstate(divide="ignore", invalid="ignore"):
            terms = np.where(cross, self.rho[None] * t * t / np.where(valid, np.abs(den), 1.0), 0.0)
        if self.cell > 0:
            I, S = self.importance(X)
            terms = terms * (I[:, self.cell_of] / S[:, None])
        # margins, as the tracer takes them
        oinf = np.abs(X).max(axis=1)[:, None]
        tabs = np.minimum(np.where(valid, np.abs(t), 0.0), 1e6)
        dxe = eX[:, None] + tabs * ew[:, None] + KAPPA * UGEOM * (oinf + self.pmax[None, :] + tabs)
        dte = np.minimum(dxe / np.maximum(np.abs(den), 1e-12), 1e6)
        duv = dte / self.smin[None, :]
        dq2 = 2.0 * np.sqrt(q2) * duv + duv * duv + KAPPA * UGEOM * k2
        amb = np.any(valid & (t > -dte) & (np.abs(q2 - k2) <= dq2), axis=1)
        amb |= np.any(valid & (q2 <= k2 + dq2) & (np.abs(t) <= dte), axis=1)
        return terms.sum(axis=1), amb


def path_trace_nee(scene, cam, prm, em=None, pixels=None, samples=None):
    """Per-(pixel, sample) path values of the MIS estimator, as
    render.path_trace: dict value [M,S,3], flags [M,S], nseg [M,S] (segments
    traced, light segments included)."""
    sc = scene if isinstance(scene, Scene64) else Scene64(scene)
    if em is None:
        em = Emitters(sc, prm.tau_E, prm.k_sigma)
    assert not prm.additive, "the MIS estimator is defined for the emitter-terminated path tracer"
    pix, _, _ = _pixels(cam, pixels)
    samples = np.arange(prm.spp) if samples is None else np.asarray(list(samples), dtype=np.int64)
    M, S = pix.size, samples.size
    rows = np.repeat(np.arange(M), S)
    sidx = np.tile(np.arange(S), M)
    P_pix = pix[rows]
    P_smp = samples[sidx]
    npaths = rows.size
    value = np.zeros((npaths, 3))
    flags = np.zeros(npaths, dtype=np.int64)
    nseg = np.zeros(npaths, dtype=np.int64)
    beta = np.ones((npaths, 3))
    pb_prev = np.zeros(npaths)          # cosine pdf of the direction that made the current segment
    O = np.zeros((npaths, 3))
    W = np.zeros((npaths, 3))
    for s_ in np.unique(P_smp):
        sel = P_smp == s_
        o, w = _camera(cam, P_pix[sel], P_pix[sel] % cam.width, P_pix[sel] // cam.width, int(s_), prm)
        O[sel], W[sel] = o, w
    eO = np.zeros(npaths)
    ew = np.zeros(npaths)
    tau = prm.tau_E
    alive = np.arange(npaths)
    k = 0
    while alive.size:
        segs = trace(sc, O[alive], W[alive], prm, eO=eO[alive], ew=ew[alive], seg_k=k)
        nxt, newO, newW, neO, new_ = [], [], [], [], []
        refl = []
        emit = [j for j, sg in enumerate(segs) if sg.hit and sg.E > tau]
        wts = np.ones(len(segs))
        if k >= 1 and emit:
            ps = alive[emit]
            pl, amb = em.pdf(O[ps], W[ps], eO[ps], ew[ps])
            pb = pb_prev[ps]
            den = pb * pb + pl * pl
            wts[emit] = np.where(den > 0.0, pb * pb / np.where(den > 0.0, den, 1.0), 1.0)
            flags[ps[amb]] |= F_NEE
        for j, sg in enumerate(segs):
            p = alive[j]
            nseg[p] += 1
            flags[p] |= sg.flags
            if not sg.hit:
                continue
            if sg.E > tau:
                value[p] += beta[p] * sg.R * wts[j]
                continue
            if k == prm.max_depth:
                continue
            refl.append(j)
        if refl:
            refl = np.array(refl)
            ps = alive[refl]
            Nt = np.array([segs[j].Nt for j in refl])
            Dt = np.array([segs[j].Dt for j in refl])
            Pv = np.array([segs[j].P for j in refl])
            eX = np.array([segs[j].eX for j in refl])
            ewb = np.array([segs[j].ew for j in refl])
            beta[ps] *= Pv
            Xo = O[ps] + Dt[:, None] * W[ps]
            # ---- light sample (before Russian roulette)
            if em.count:
                v0, v1, v2, v3 = philox.uniforms(P_pix[ps], P_smp[ps], NEE_SEGMENT + k, prm.camera_id, prm.seed)
                _, y, amb = em.sample(v0, v1, v2, v3, Xo, eX)
                dl = y - Xo
                dist = np.linalg.norm(dl, axis=1)
                Wl = dl / dist[:, None]
                cl = np.einsum("mc,mc->m", Wl, Nt)
                ewl = (eX + KAPPA * UGEOM * (np.abs(y).max(axis=1) + np.abs(Xo).max(axis=1))) / dist + KAPPA * UGEOM
                amb |= np.abs(cl) <= ewb + ewl + KAPPA * UGEOM
                flags[ps[amb]] |= F_NEE
                up = np.nonzero(cl > 0.0)[0]
                if up.size:
                    lsegs = trace(sc, Xo[up], Wl[up], prm, eO=eX[up], ew=ewl[up], seg_k=k + 1)
                    pl, pamb = em.pdf(Xo[up], Wl[up], eX[up], ewl[up])
                    pb = cl[up] / np.pi
                    for jj, ls in enumerate(lsegs):
                        p = ps[up[jj]]
                        nseg[p] += 1
                        flags[p] |= ls.flags | (F_NEE if pamb[jj] else 0)
                        if ls.hit and ls.E > tau:
                            value[p] += beta[p] * ls.R * (pb[jj] * pl[jj] / (pb[jj] ** 2 + pl[jj] ** 2))
            # ---- cosine sample, Russian roulette, as the plain path tracer
            u0, u1, u2, _ = philox.uniforms(P_pix[ps], P_smp[ps], k, prm.camera_id, prm.seed)
            Wd = cosine_direction(Nt, u0, u1)
            pb_prev[ps] = np.maximum(np.einsum("mc,mc->m", Wd, Nt), 0.0) / np.pi
            keep = np.ones(ps.size, dtype=bool)
            if prm.rr_start > 0 and k + 1 >= prm.rr_start:
                q = np.minimum(0.95, beta[ps].max(axis=1))
                keep = u2 < q
                close = np.abs(u2 - q) <= q * (k + 1) * 8 * UF32 + 1e-7
                flags[ps[close]] |= F_RR
                beta[ps[keep]] /= q[keep][:, None]
            for jj, j in enumerate(refl):
                if keep[jj]:
                    nxt.append(alive[j])
                    newO.append(Xo[jj])
                    newW.append(Wd[jj])
                    neO.append(segs[j].eX)
                    new_.append(segs[j].ew)
        alive = np.array(nxt, dtype=np.int64)
        if alive.size:
            O[alive] = np.array(newO)
            W[alive] = np.array(newW)
            eO[alive] = np.array(neO)
            ew[alive] = np.array(new_)
        k += 1
    return dict(value=value.reshape(M, S, 3), flags=flags.reshape(M, S), nseg=nseg.reshape(M, S),
                pixels=pix, samples=samples)


__all__ = ["Emitters", "path_trace_nee", "NEE_SEGMENT", "F_NEE"]
