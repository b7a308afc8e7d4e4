"""Renderers on top of the brute-force tracer, float64.

* zero_bounce: the radiant-scene image L_o^0 = R along the camera ray
  (Sec. 3.2, "Radiance Loss").
* single_bounce: emission-aware single bounce (Sec. 3.3, Eq. 5-7). The
  camera ray is traced once per pixel through the pixel centre. Miss -> 0;
  E > tau_E -> R (emitters do not reflect, Eq. 5); otherwise
  L = P * (1/n_spp) sum_s R(w'_s), where w'_s is cosine-sampled about Nt from
  the bounce point X = O + Dt w (Sec. 3.1, "Light Bouncing") and R(w'_s) is
  the composited radiance of every surfel on the secondary ray (the radiance
  cache, no emitter test). With f = P/pi and pdf cos/pi, f cos / pdf = P.
* path_trace: Eq. 9. Per sample: throughput beta = 1; at segment k: miss ->
  0; E > tau_E -> add beta*R and stop; k == max_depth -> discard (0);
  otherwise beta *= P, sample w' with Philox counter (pixel, sample, k, id),
  move to X and continue. Russian roulette (an addition, not in the paper)
  applies when the new depth k+1 >= rr_start > 0: q = min(0.95, max_c beta_c),
  the path survives iff u2 < q, and beta /= q. Test-only additive mode adds
  beta*R at every hit and always reflects (the first line of Eq. 5).

Pinned by tests/test_oracle_render.py: white furnace (closed form
E * sum_k (A rho)^k -> E / (1 - rho)), a quadrature of the single-bounce
integral for one emitter over one receiver (scipy dblquad), the identities
PT(max_depth=0) = emitter part of the 0-bounce image and PT(max_depth=1) =
single bounce where the secondary segment is an emitter, linearity in
radiance, and rho = 0 giving the direct-emitter image.
"""
import numpy as np

from . import philox
from .frames import camera_rays, cosine_direction
from .tracer import Scene64, trace, F_RR, UF32

JITTER_SEGMENT = 0xFFFFFFFF


def _pixels(cam, pixels):
    if pixels is None:
        pix = np.arange(cam.width * cam.height, dtype=np.int64)
    else:
        pix = np.asarray(pixels, dtype=np.int64)
    return pix, pix % cam.width, pix // cam.width


def _camera(cam, pix, px, py, sample, prm):
    jit = None
    if prm.jitter:
        u0, u1, _, _ = philox.uniforms(pix, sample, JITTER_SEGMENT, prm.camera_id, prm.seed)
        jit = (u0, u1)
    return camera_rays(cam, px, py, jit)


def zero_bounce(scene, cam, prm, pixels=None):
    sc = scene if isinstance(scene, Scene64) else Scene64(scene)
    pix, px, py = _pixels(cam, pixels)
    O, W = _camera(cam, pix, px, py, 0, prm)
    segs = trace(sc, O, W, prm)
    return np.array([s.R for s in segs]), segs


def single_bounce(scene, cam, prm, pixels=None, keep_segments=False):
    """Returns dict: L [M,3], branch [M] (0 miss, 1 emit, 2 reflect),
    flags [M], R1 [M,spp,3] (zero where not traced), camera segments, and
    optionally the secondary segments [M][spp]."""
    sc = scene if isinstance(scene, Scene64) else Scene64(scene)
    pix, px, py = _pixels(cam, pixels)
    M, S = pix.size, prm.spp
    O, W = _camera(cam, pix, px, py, 0, prm)
    cam_segs = trace(sc, O, W, prm, seg_k=0)
    L = np.zeros((M, 3))
    branch = np.zeros(M, dtype=np.int64)
    flags = np.array([s.flags for s in cam_segs], dtype=np.int64)
    R1 = np.zeros((M, S, 3))
    sec = [[None] * S for _ in range(M)] if keep_segments else None
    refl = []
    for i, s in enumerate(cam_segs):
        if not s.hit:
            continue
        if s.E > prm.tau_E:
            branch[i] = 1
            L[i] = s.R
        else:
            branch[i] = 2
            refl.append(i)
    if refl:
        refl = np.array(refl)
        rows = np.repeat(refl, S)
        samp = np.tile(np.arange(S), refl.size)
        u0, u1, _, _ = philox.uniforms(pix[rows], samp, 0, prm.camera_id, prm.seed)
        Nt = np.array([cam_segs[i].Nt for i in rows])
        Dt = np.array([cam_segs[i].Dt for i in rows])
        X = O[rows] + Dt[:, None] * W[rows]
        Wd = cosine_direction(Nt, u0, u1)
        eX = np.array([cam_segs[i].eX for i in rows])
        ew = np.array([cam_segs[i].ew for i in rows])
        segs = trace(sc, X, Wd, prm, eO=eX, ew=ew, seg_k=1)
        for j, sg in enumerate(segs):
            i, s_ = rows[j], samp[j]
            R1[i, s_] = sg.R
            flags[i] |= sg.flags & ~0   # any flag on a secondary flags the pixel
            if keep_segments:
                sec[i][s_] = sg
        for i in refl:
            L[i] = cam_segs[i].P * R1[i].mean(axis=0)
    out = dict(L=L, branch=branch, flags=flags, R1=R1, cam=cam_segs, pixels=pix, O=O, W=W)
    if keep_segments:
        out["sec"] = sec
    return out


def path_trace(scene, cam, prm, pixels=None, samples=None, keep_segments=False):
    """Per-(pixel, sample) path values. pixels: [M] linear pixel ids;
    samples: iterable of sample indices (default range(spp)).
    Returns dict: value [M,S,3], flags [M,S], nseg [M,S], optionally the
    per-path segment lists."""
    sc = scene if isinstance(scene, Scene64) else Scene64(scene)
    pix, px, py = _pixels(cam, pixels)
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
    segs_out = [[] for _ in range(npaths)] if keep_segments else None
    # camera rays (jitter, if on, depends on the sample)
    O = np.zeros((npaths, 3))
    W = np.zeros((npaths, 3))
    for s_ in np.unique(P_smp):
        sel = P_smp == s_
        o, w = _camera(cam, P_pix[sel], P_pix[sel] % cam.width, P_pix[sel] // cam.width, int(s_), prm)
        O[sel], W[sel] = o, w
    eO = np.zeros(npaths)
    ew = np.zeros(npaths)
    alive = np.arange(npaths)
    k = 0
    while alive.size:
        segs = trace(sc, O[alive], W[alive], prm, eO=eO[alive], ew=ew[alive], seg_k=k)
        nxt = []
        newO, newW, neO, new_ = [], [], [], []
        refl = []
        for j, sg in enumerate(segs):
            p = alive[j]
            nseg[p] += 1
            flags[p] |= sg.flags
            if keep_segments:
                segs_out[p].append(sg)
            if not sg.hit:
                continue
            if prm.additive:
                value[p] += beta[p] * sg.R
            elif sg.E > prm.tau_E:
                value[p] += beta[p] * sg.R
                continue
            if k == prm.max_depth:
                continue
            refl.append(j)
        if refl:
            refl = np.array(refl)
            ps = alive[refl]
            u0, u1, u2, _ = philox.uniforms(P_pix[ps], P_smp[ps], k, prm.camera_id, prm.seed)
            Nt = np.array([segs[j].Nt for j in refl])
            Dt = np.array([segs[j].Dt for j in refl])
            Pv = np.array([segs[j].P for j in refl])
            beta[ps] *= Pv
            Xo = O[ps] + Dt[:, None] * W[ps]
            Wd = cosine_direction(Nt, u0, u1)
            keep = np.ones(ps.size, dtype=bool)
            if prm.rr_start > 0 and k + 1 >= prm.rr_start:
                q = np.minimum(0.95, beta[ps].max(axis=1))
                keep = u2 < q
                # margin: a float32 throughput carries a few ulps per product
                close = np.abs(u2 - q) <= q * (k + 1) * 8 * UF32 + 1e-7
                flags[ps[close]] |= F_RR
                beta[ps[keep]] /= q[keep][:, None]
            for jj, j in enumerate(refl):
                if keep[jj]:
                    p = alive[j]
                    nxt.append(p)
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
    out = dict(value=value.reshape(M, S, 3), flags=flags.reshape(M, S), nseg=nseg.reshape(M, S),
               pixels=pix, samples=samples)
    if keep_segments:
        out["segments"] = [segs_out[r * S:(r + 1) * S] for r in range(M)]
    return out
