"""Ray-surfel intersection, ordering and compositing, float64, brute force.

Definitions followed (Sec. 3.1, "2D Gaussian Ray Tracing", Eq. 1-3):

* A ray O + t w meets a surfel on its tangent plane (the plane through p
  with normal n = t_u x t_v): den = w.n, t = ((p - O).n) / den, local offset
  y = O + t w - p, coordinates u = y.t_u / s_u, v = y.t_v / s_v.
  Readings: rejected if |den| <= 1e-12 or opacity == 0; accepted iff
  t > t_min and u^2 + v^2 <= k_sigma^2.
* Response g = exp(-(u^2 + v^2) / 2) (Eq. 1); alpha = opacity * g, with no
  clamp.
* Accepted hits are visited in ascending order of the key
  (floor(t / dq), index) (dq = 0: (t, index)).
* Front-to-back blending (Eq. 2): w_i = T_{i-1} alpha_i, T_i = T_{i-1}(1 -
  alpha_i), T_0 = 1, stopping after the first hit whose T_i < T_min.
* Traced quantities (Eq. 3): N = sum w_i n'_i with n'_i = -sign(w.n_i) n_i
  (the normal turned toward the ray origin), D = sum w_i t_i, R = sum w_i r_i,
  E = sum w_i e_i, P = sum w_i rho_i; A = 1 - T_last; Nt = N / |N|,
  Dt = D / A. A segment misses iff A == 0.

Pinned by tests/test_oracle_trace.py: a single surfel's analytic hit (t, u,
v, g and every traced quantity in closed form), the compositing identities
(weights plus final transmittance sum to one, constant quantity gives
V = A v, transmittance independent of order, split associativity), and a
pure-Python per-ray loop on tiny scenes.

Decision margins. Besides the exact result, each segment carries flag bits
for decisions that another evaluation of the same definition, with
different rounding, may take differently: a surfel near its acceptance rim
or near t_min, a key near a bucket edge, transmittance near T_min at the
stopping hit, E near tau_E, a nearly empty segment and a near-singular
hemisphere frame. Each margin is an error bound built from a rounding model
(unit roundoff UGEOM for ray geometry, which a float32 evaluation would
set to 2^-24 and a double-precision one to 2^-53, times a safety factor
KAPPA, times the magnitudes involved; UF32 for quantities kept in float32),
plus the propagated error of the ray's own origin and direction, which the
renderers carry from segment to segment. Flagged segments are excluded from
bit-exact comparisons and counted.
"""
import numpy as np

from .frames import quat_frames, hemisphere_frame

UGEOM = 2.0 ** -53      # ray geometry evaluated in double precision
UF32 = 2.0 ** -24       # quantities stored in float32 (E against tau_E, throughput)
KAPPA = 64.0

F_RIM, F_TMIN, F_BUCKET, F_TERM, F_EMIT, F_THIN, F_FRAME, F_PAR, F_RR = (1 << i for i in range(9))
FLAG_NAMES = {F_RIM: "rim", F_TMIN: "tmin", F_BUCKET: "bucket", F_TERM: "term", F_EMIT: "emit",
              F_THIN: "thin", F_FRAME: "frame", F_PAR: "parallel", F_RR: "rr"}


class Scene64:
    """float64 copy of a float32 surfel scene (exact upcast) with frames."""

    def __init__(self, scene):
        a = scene.arrays() if hasattr(scene, "arrays") else scene
        self.p = np.asarray(a["pos"], dtype=np.float64).T.copy()
        self.tu, self.tv, self.n = quat_frames(a["rot"])
        s = np.asarray(a["scale"], dtype=np.float64)
        self.su, self.sv = s[0].copy(), s[1].copy()
        self.sigma = np.asarray(a["opacity"], dtype=np.float64).copy()
        self.rho = np.asarray(a["albedo"], dtype=np.float64).T.copy()
        self.r = np.asarray(a["radiance"], dtype=np.float64).T.copy()
        self.e = np.asarray(a["emissive"], dtype=np.float64).copy()
        self.pmax = np.abs(self.p).max(axis=1)
        self.smin = np.minimum(self.su, self.sv)
        self.N = self.p.shape[0]


class Segment:
    """Result of tracing one ray segment."""
    __slots__ = ("hits", "t", "alpha", "n_acc", "N", "D", "R", "E", "P", "A", "Nt", "Dt", "Nlen",
                 "T", "flags", "eX", "ew", "mlen", "O", "W")

    def __init__(self):
        self.hits = np.zeros(0, dtype=np.int64)
        self.t = np.zeros(0)
        self.alpha = np.zeros(0)
        self.n_acc = 0
        self.N = np.zeros(3)
        self.D = 0.0
        self.R = np.zeros(3)
        self.E = 0.0
        self.P = np.zeros(3)
        self.A = 0.0
        self.T = 1.0
        self.Nt = np.zeros(3)
        self.Dt = 0.0
        self.Nlen = 0.0
        self.flags = 0
        self.eX = 0.0
        self.ew = 0.0
        self.mlen = 1.0
        self.O = None
        self.W = None

    @property
    def hit(self) -> bool:
        return self.A > 0.0


def _batch_size(n):
    return max(1, (1 << 20) // max(n, 1))


def trace(sc: Scene64, O, W, prm, eO=None, ew=None, seg_k=0):
    """Trace rays O [M,3], W [M,3] (unit) through every surfel.

    eO, ew: per-ray absolute origin error and direction error (radians)
    bounds used only for the margin flags. Returns a list of Segment."""
    O = np.atleast_2d(np.asarray(O, dtype=np.float64))
    W = np.atleast_2d(np.asarray(W, dtype=np.float64))
    M = O.shape[0]
    eO = np.zeros(M) if eO is None else np.broadcast_to(np.asarray(eO, dtype=np.float64), (M,))
    ew = np.zeros(M) if ew is None else np.broadcast_to(np.asarray(ew, dtype=np.float64), (M,))
    out = []
    B = _batch_size(sc.N)
    for b0 in range(0, M, B):
        out.extend(_trace_batch(sc, O[b0:b0 + B], W[b0:b0 + B], prm, eO[b0:b0 + B], ew[b0:b0 + B], seg_k))
    return out


def _trace_batch(sc, O, W, prm, eO, ew, seg_k):
    k2 = prm.k_sigma * prm.k_sigma
    px, py, pz = (sc.p[:, c][None, :] for c in range(3))
    nx, ny, nz = (sc.n[:, c][None, :] for c in range(3))
    ox, oy, oz = (O[:, c][:, None] for c in range(3))
    wx, wy, wz = (W[:, c][:, None] for c in range(3))
    dx, dy, dz = px - ox, py - oy, pz - oz                 # d = p - O
    den = wx * nx + wy * ny + wz * nz                      # w . n
    num = dx * nx + dy * ny + dz * nz                      # (p - O) . n
    valid = (np.abs(den) > 1e-12) & (sc.sigma[None, :] > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(valid, num / np.where(valid, den, 1.0), np.inf)
    yx, yy, yz = t * wx - dx, t * wy - dy, t * wz - dz     # y = O + t w - p
    yx = np.where(valid, yx, 0.0)
    yy = np.where(valid, yy, 0.0)
    yz = np.where(valid, yz, 0.0)
    u = (yx * sc.tu[:, 0][None] + yy * sc.tu[:, 1][None] + yz * sc.tu[:, 2][None]) / sc.su[None]
    v = (yx * sc.tv[:, 0][None] + yy * sc.tv[:, 1][None] + yz * sc.tv[:, 2][None]) / sc.sv[None]
    q2 = u * u + v * v
    acc = valid & (t > prm.t_min) & (q2 <= k2)

    # rounding-error model for the margin flags (UGEOM: ray geometry in double
    # precision, times KAPPA): dxe bounds the absolute error
    # of a hit point, dte its distance along the ray, duv its tangent-plane
    # coordinates (the hit point slides by dxe / |cos| within the plane)
    oinf = np.abs(O).max(axis=1)[:, None]
    tabs = np.minimum(np.where(valid, np.abs(t), 0.0), 1e6)
    dxe = eO[:, None] + tabs * ew[:, None] + KAPPA * UGEOM * (oinf + sc.pmax[None, :] + tabs)
    acos = np.maximum(np.abs(den), 1e-12)
    dte = np.minimum(dxe / acos, 1e6)
    duv = dte / sc.smin[None, :]
    dq2 = 2.0 * np.sqrt(q2) * duv + duv * duv + KAPPA * UGEOM * k2
    near_t = valid & (t > prm.t_min - dte)
    rim = np.any(near_t & (np.abs(q2 - k2) <= dq2), axis=1)
    tmin = np.any(valid & (q2 <= k2 + dq2) & (np.abs(t - prm.t_min) <= dte), axis=1)
    par = np.any(valid & (q2 <= k2 + dq2) & (t > prm.t_min - dte) & (np.abs(den) < 1e-6), axis=1)

    res = []
    for b in range(O.shape[0]):
        seg = Segment()
        seg.O, seg.W = O[b], W[b]
        idx = np.nonzero(acc[b])[0]
        flags = (F_RIM if rim[b] else 0) | (F_TMIN if tmin[b] else 0) | (F_PAR if par[b] else 0)
        if idx.size == 0:
            seg.flags = flags
            seg.eX = eO[b]
            seg.ew = ew[b]
            res.append(seg)
            continue
        tb = t[b, idx]
        if prm.depth_quantum > 0:
            bucket = np.floor(tb / prm.depth_quantum)
            order = np.lexsort((idx, bucket))
        else:
            order = np.lexsort((idx, tb))
        idx, tb = idx[order], tb[order]
        alpha = sc.sigma[idx] * np.exp(-0.5 * q2[b, idx])
        T = np.cumprod(1.0 - alpha)
        below = np.nonzero(T < prm.T_min)[0]
        m = int(below[0]) if below.size else idx.size - 1
        terminated = below.size > 0
        Tprev = np.concatenate([[1.0], T[:-1]])
        wts = Tprev[:m + 1] * alpha[:m + 1]
        hi = idx[:m + 1]
        den_h = den[b, hi]
        nprime = -np.sign(den_h)[:, None] * sc.n[hi]
        seg.hits = hi
        seg.t = tb[:m + 1]
        seg.alpha = alpha[:m + 1]
        seg.n_acc = int(idx.size)
        seg.N = (wts[:, None] * nprime).sum(axis=0)
        seg.D = float((wts * seg.t).sum())
        seg.R = (wts[:, None] * sc.r[hi]).sum(axis=0)
        seg.E = float((wts * sc.e[hi]).sum())
        seg.P = (wts[:, None] * sc.rho[hi]).sum(axis=0)
        seg.T = float(T[m])
        seg.A = 1.0 - seg.T
        seg.Nlen = float(np.linalg.norm(seg.N))
        seg.Nt = seg.N / seg.Nlen
        seg.Dt = seg.D / seg.A

        # --- ordering margin
        dte_h = dte[b, idx]
        tcut = tb[m] + (prm.depth_quantum if prm.depth_quantum > 0 else 0.0) + dte_h[m]
        win = tb <= tcut
        if prm.depth_quantum > 0:
            # a key that may fall in the neighbouring bucket changes the order
            # only if another hit sits in the same or an adjacent bucket
            bk = np.floor(tb / prm.depth_quantum)
            fr = tb / prm.depth_quantum - bk
            edge = np.minimum(fr, 1.0 - fr) * prm.depth_quantum
            amb = win & (edge <= dte_h)
            if np.any(amb):
                close = np.zeros(tb.size, dtype=bool)
                if tb.size > 1:
                    near = np.diff(bk) <= 1
                    close[1:] |= near
                    close[:-1] |= near
                if np.any(amb & close):
                    flags |= F_BUCKET
        else:
            tw, ew_ = tb[win], dte_h[win]
            if tw.size > 1 and np.any(np.diff(tw) <= ew_[1:] + ew_[:-1]):
                flags |= F_BUCKET
        # --- termination margin: relative alpha error ea, weight error dw
        ea = np.sqrt(q2[b, hi]) * duv[b, hi] + 4 * KAPPA * UGEOM
        lt = alpha[:m + 1] / (1.0 - alpha[:m + 1]) * ea
        dlnT = float(np.sum(lt)) + (m + 1) * KAPPA * UGEOM
        lnTmin = np.log(prm.T_min)
        if terminated:
            if abs(np.log(T[m]) - lnTmin) <= dlnT or (m >= 1 and abs(np.log(T[m - 1]) - lnTmin) <= dlnT):
                flags |= F_TERM
        elif abs(np.log(max(T[m], 1e-300)) - lnTmin) <= dlnT:
            flags |= F_TERM
        dw = ea + np.concatenate([[0.0], np.cumsum(lt)[:-1]])
        dE = float(np.sum(wts * sc.e[hi] * dw)) + 4 * UF32 * max(seg.E, prm.tau_E)
        if abs(seg.E - prm.tau_E) <= dE:
            flags |= F_EMIT
        if seg.A < 1e-4:
            flags |= F_THIN
        _, _, mlen = hemisphere_frame(seg.Nt[None, :])
        seg.mlen = float(mlen[0])
        if seg.mlen < 1e-3:
            flags |= F_FRAME
        # --- error carried to the next segment: Dt and Nt are weighted means,
        # so weight errors move them by the spread of the averaged values
        dDt = float(np.sum(wts * (np.abs(seg.t - seg.Dt) * dw + dte[b, hi]))) / seg.A
        eN = float(np.sum(wts * np.linalg.norm(nprime - seg.Nt[None, :], axis=1) * dw)) / max(seg.Nlen, 1e-300)
        eN += KAPPA * UGEOM
        seg.eX = eO[b] + abs(seg.Dt) * ew[b] + dDt + KAPPA * UGEOM * (oinf[b, 0] + 2 * abs(seg.Dt))
        seg.ew = eN * (1.0 + 2.0 / max(seg.mlen, 1e-3)) + KAPPA * UGEOM
        seg.flags = flags
        res.append(seg)
    return res


def composite_list(alpha, values, T_min):
    """Plain front-to-back blending of a given ordered hit list (Eq. 2): returns
    (V, weights, T list, stop index). Used by the pins and by the per-ray
    reference loop."""
    T = 1.0
    V = np.zeros(np.asarray(values).shape[1:]) if np.ndim(values) > 1 else 0.0
    ws, Ts = [], []
    stop = len(alpha) - 1
    for i, a in enumerate(alpha):
        w = T * a
        V = V + w * np.asarray(values[i])
        T = T * (1.0 - a)
        ws.append(w)
        Ts.append(T)
        if T < T_min:
            stop = i
            break
    return V, np.array(ws), np.array(Ts), stop
