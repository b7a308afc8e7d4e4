"""Stage-0 radiant-scene objective (Sec. 3.2, Eq. 4), torch.float64 on the
CPU, differentiated by autograd.

Images, per pixel of a camera (one ray through the pixel centre, as in the
0-bounce render): the camera segment's Nt = N/|N|, Dt = D/A, R and E
(Sec. 3.1, Eq. 3), on the hit lists that the float64 forward pass
(render.zero_bounce) fixed; a pixel whose ray blends nothing is a miss and
has all four at 0.

Objective (Eq. 4), with weights (lc, ln, ld, le):
  lc * mean over pixels and channels of |PQ(R) - PQ(R_gt)|        (L_c^0)
  ln * mean over hit pixels of (1 - Nt . N_mono)                  (L_n)
  ld * mean over valid pixels of (1 - N_d . N_mono)               (L_d)
  le * mean over pixels of |E - M|                                (L_e)
N_d is the distance normal, the normal of the surface that the depth map
describes: with X(x, y) = O + Dt W the pixel's point,
N_d = normalize((X(x+1, y) - X(x-1, y)) x (X(x, y+1) - X(x, y-1))), turned to
face the camera (N_d . W <= 0). A pixel is valid for L_d when it and its
four neighbours are inside the image and hit.

Readings (the paper leaves these open): L_c is the L1 term of the colour
loss on PQ-encoded values (as in bake.py; the D-SSIM term is left out); the
norm of L_n, L_d and L_e is the mean over the pixels that carry the term;
the distance normal uses central differences of the back-projected points
(the image-space gradient of Dt); the orientation flip is a discrete
decision held fixed, like the hit lists.

Functions:
  stage0_images(scene, cam, prm)            images and the forward segments
  stage0_objective(...)                     loss, parameter gradients (pos,
                                            rot, scale, opacity, radiance,
                                            emissive), image gradients
  image_objective(images, targets, ...)     the loss as a function of the
                                            images alone, and its gradient
  images_vjp(scene, cam, prm, d_images)     parameter gradients of a linear
                                            function of the images

Pinned by tests/test_oracle_stage0.py: closed forms for one surfel seen
head-on (Nt = n facing the camera, Dt = t, R = alpha r, E = alpha e); the
distance normal of a tilted plane equals the plane's normal; central
differences of the float64 forward on random parameters with an unchanged
discrete signature; central differences of the image objective; the
chain rule stage0_objective = images_vjp(image gradients).
"""
import numpy as np
import torch

from .bake import pq, pq_grad
from .grad import _frames, _pad, _segment
from .render import zero_bounce
from .tracer import Scene64

STAGE0_PARAMS = ("pos", "rot", "scale", "opacity", "radiance", "emissive")


def _pq_t(L):
    """PQ with the slope of bake.pq_grad (taken at max(Y, 2^-24)): the value
    is pq(L) and the derivative pq_grad(L)."""
    Ld = L.detach()
    value = torch.as_tensor(pq(Ld.numpy()))
    slope = torch.as_tensor(pq_grad(Ld.numpy()))
    return value + slope * (L - Ld)


def stage0_images(scene, cam, prm):
    """numpy images (Nt [M,3], Dt [M], R [M,3], E [M], hit [M]) and the
    forward segments of all pixels."""
    sc = scene if isinstance(scene, Scene64) else Scene64(scene)
    _, segs = zero_bounce(sc, cam, prm)
    M = len(segs)
    out = {"Nt": np.zeros((M, 3)), "Dt": np.zeros(M), "R": np.zeros((M, 3)), "E": np.zeros(M),
           "hit": np.zeros(M, dtype=bool)}
    for i, s in enumerate(segs):
        if s.hits.size and s.A > 0:
            out["Nt"][i], out["Dt"][i], out["R"][i], out["E"][i] = s.Nt, s.Dt, s.R, s.E
            out["hit"][i] = True
    return out, segs


def _neighbours(cam):
    W, H = cam.width, cam.height
    pix = np.arange(W * H)
    x, y = pix % W, pix // W
    inside = (x > 0) & (x < W - 1) & (y > 0) & (y < H - 1)
    xm, xp = np.clip(x - 1, 0, W - 1), np.clip(x + 1, 0, W - 1)
    ym, yp = np.clip(y - 1, 0, H - 1), np.clip(y + 1, 0, H - 1)
    return inside, y * W + xm, y * W + xp, ym * W + x, yp * W + x


def _objective(Nt, Dt, R, E, hit, O, Wd, targets, weights, cam, flip=None):
    """Eq. 4 on torch image tensors; returns (loss, flip) where flip holds
    the orientation decisions of the distance normals."""
    lc, ln, ld, le = weights
    M = Nt.shape[0]
    rgb_gt = torch.as_tensor(np.asarray(targets["rgb"], dtype=np.float64).reshape(M, 3))
    n_mono = torch.as_tensor(np.asarray(targets["normal"], dtype=np.float64).reshape(M, 3))
    mask = torch.as_tensor(np.asarray(targets["mask"], dtype=np.float64).reshape(M))
    hit_t = torch.as_tensor(hit)
    loss = lc * (_pq_t(R) - _pq_t(rgb_gt)).abs().mean()
    if hit.any():
        loss = loss + ln * (1.0 - (Nt[hit_t] * n_mono[hit_t]).sum(1)).mean()
    loss = loss + le * (E - mask).abs().mean()
    inside, l, r, u, d = _neighbours(cam)
    valid = inside & hit & hit[l] & hit[r] & hit[u] & hit[d]
    if valid.any():
        X = O + Dt[:, None] * Wd
        v = torch.as_tensor(np.nonzero(valid)[0])
        ex = X[torch.as_tensor(r)[v]] - X[torch.as_tensor(l)[v]]
        ey = X[torch.as_tensor(d)[v]] - X[torch.as_tensor(u)[v]]
        c = torch.linalg.cross(ex, ey, dim=1)
        nd = c / torch.linalg.norm(c, dim=1, keepdim=True)
        if flip is None:
            flip = ((nd.detach() * Wd[v]).sum(1) > 0).numpy()
        nd = torch.where(torch.as_tensor(flip)[:, None], -nd, nd)
        loss = loss + ld * (1.0 - (nd * n_mono[v]).sum(1)).mean()
    return loss, flip


def image_objective(images, targets, weights, cam, prm):
    """Eq. 4 as a function of the images (the hit mask fixed): returns the
    loss and its gradient with respect to Nt [M,3], Dt [M], R [M,3], E [M]."""
    sc_rays = _rays(cam, prm)
    t = {k: torch.tensor(np.asarray(images[k], dtype=np.float64), requires_grad=True) for k in ("Nt", "Dt", "R", "E")}
    loss, _ = _objective(t["Nt"], t["Dt"], t["R"], t["E"], np.asarray(images["hit"]), *sc_rays, targets, weights, cam)
    loss.backward()
    return float(loss.detach()), {k: (t[k].grad.numpy().copy() if t[k].grad is not None else np.zeros(t[k].shape))
                                  for k in t}


def _rays(cam, prm):
    from .render import _camera, _pixels
    pix, px, py = _pixels(cam, None)
    O, W = _camera(cam, pix, px, py, 0, prm)
    return torch.from_numpy(O), torch.from_numpy(W)


def _images_t(th, segs, images, O, Wd):
    fr = _frames(th["rot"])
    idx, mask = _pad([s.hits for s in segs])
    den0 = (Wd[:, None, :] * fr[2].detach()[idx]).sum(-1)
    sign = torch.where(mask, -torch.sign(den0), torch.zeros_like(den0))
    N, D, R, E, _, A = _segment(th, fr, O, Wd, idx, mask, sign)
    h = torch.as_tensor(np.asarray(images["hit"]))
    one = torch.ones_like(A)
    Nl = torch.linalg.norm(torch.where(h[:, None], N, torch.ones_like(N)), dim=1)   # (no 0/0 at misses)
    Nt = torch.where(h[:, None], N / Nl[:, None], torch.zeros_like(N))
    Dt = torch.where(h, D / torch.where(h, A, one), torch.zeros_like(D))
    R = torch.where(h[:, None], R, torch.zeros_like(R))
    E = torch.where(h, E, torch.zeros_like(E))
    return Nt, Dt, R, E


def _theta(scene):
    a = scene.arrays() if hasattr(scene, "arrays") else scene
    return {k: torch.tensor(np.asarray(a[k], dtype=np.float64), requires_grad=(k in STAGE0_PARAMS))
            for k in ("pos", "rot", "scale", "opacity", "albedo", "radiance", "emissive")}


def _grads(th):
    return {k: (th[k].grad.numpy().copy() if th[k].grad is not None else np.zeros(th[k].shape))
            for k in STAGE0_PARAMS}


def images_vjp(scene, cam, prm, d_images, fwd=None):
    """Parameter gradients of sum over pixels of d_images . (Nt, Dt, R, E)
    (d_images: dict of arrays shaped like the images)."""
    sc = scene if isinstance(scene, Scene64) else Scene64(scene)
    if fwd is None:
        fwd = stage0_images(sc, cam, prm)
    images, segs = fwd
    th = _theta(scene)
    O, Wd = _rays(cam, prm)
    imgs = _images_t(th, segs, images, O, Wd)
    total = sum((t * torch.as_tensor(np.asarray(d_images[k], dtype=np.float64))).sum()
                for k, t in zip(("Nt", "Dt", "R", "E"), imgs))
    total.backward()
    return _grads(th)


def stage0_objective(scene, cam, prm, targets, weights, fwd=None):
    """Loss (Eq. 4) of the camera's images, its gradient with respect to the
    surfel parameters (component-major numpy arrays, STAGE0_PARAMS) and
    with respect to the images (Nt, Dt, R, E)."""
    sc = scene if isinstance(scene, Scene64) else Scene64(scene)
    if fwd is None:
        fwd = stage0_images(sc, cam, prm)
    images, segs = fwd
    th = _theta(scene)
    O, Wd = _rays(cam, prm)
    Nt, Dt, R, E = _images_t(th, segs, images, O, Wd)
    hit = np.asarray(images["hit"])
    for t_ in (Nt, Dt, R, E):
        t_.retain_grad()
    loss, _ = _objective(Nt, Dt, R, E, hit, O, Wd, targets, weights, cam)
    loss.backward()
    grads = _grads(th)
    dimg = {k: (v.grad.numpy().copy() if v.grad is not None else np.zeros(v.shape))
            for k, v in (("Nt", Nt), ("Dt", Dt), ("R", R), ("E", E))}
    return float(loss.detach()), grads, dimg, fwd
