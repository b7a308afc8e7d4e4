"""Gradient of the single-bounce render (Sec. 3.3, Eq. 7-8), torch.float64
on the CPU, by autograd.

The map differentiated is the single-bounce image of render.single_bounce
with every discrete decision held at the values the float64 forward pass
took: the set and order of blended hits on every segment (including the
stopping hit), the sign that turns each normal toward the ray origin, and
the branch (miss / emitter / reflect) of each pixel. Within those decisions
the image is a smooth function of the surfel parameters: centre p,
quaternion q (unnormalised), scales s_u, s_v, opacity, albedo and radiance.
The emissive term e enters only through the emitter threshold and gets no
gradient. The chain runs through the bounce point X = O + Dt w (Dt = D/A)
and the sampled direction w'(Nt, u0, u1) of the hemisphere frame, unless
detach_bounce is set, in which case X and w' are held constant (the
paper optimises albedo alone, for which the two coincide).

The formulas are those of tracer.py (Eq. 1-3) and frames.py, re-expressed on
fixed hit lists so that autograd can run; the Philox numbers are the same.

Pinned by tests/test_oracle_grad.py: central finite differences of the
float64 forward (render.single_bounce) on random parameters whose discrete
signature does not change within +-h, and closed forms for one surfel.
"""
import numpy as np
import torch

from . import philox
from .frames import HELPER
from .render import single_bounce
from .tracer import Scene64

PARAMS = ("pos", "rot", "scale", "opacity", "albedo", "radiance")


def _frames(rot):
    q = rot / torch.linalg.norm(rot, dim=0, keepdim=True)
    w, x, y, z = q
    tu = torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y + w * z), 2 * (x * z - w * y)], dim=1)
    tv = torch.stack([2 * (x * y - w * z), 1 - 2 * (x * x + z * z), 2 * (y * z + w * x)], dim=1)
    n = torch.linalg.cross(tu, tv, dim=1)
    return tu, tv, n


def _pad(lists):
    L = max([len(h) for h in lists] + [1])
    idx = np.zeros((len(lists), L), dtype=np.int64)
    mask = np.zeros((len(lists), L), dtype=bool)
    for i, h in enumerate(lists):
        idx[i, :len(h)] = h
        mask[i, :len(h)] = True
    return torch.from_numpy(idx), torch.from_numpy(mask)


def _segment(th, fr, O, W, idx, mask, sign):
    """Blend fixed hit lists: O, W [B,3]; idx, mask, sign [B,L]. Returns
    N [B,3], D [B], R [B,3], E [B], P [B,3], A [B]."""
    tu, tv, n = fr
    p = th["pos"].T[idx]
    nn = n[idx]
    d = p - O[:, None, :]
    den = (W[:, None, :] * nn).sum(-1)
    den = torch.where(mask, den, torch.ones_like(den))
    t = (d * nn).sum(-1) / den
    y = t[..., None] * W[:, None, :] - d
    u = (y * tu[idx]).sum(-1) / th["scale"][0][idx]
    v = (y * tv[idx]).sum(-1) / th["scale"][1][idx]
    alpha = torch.where(mask, th["opacity"][idx] * torch.exp(-0.5 * (u * u + v * v)), torch.zeros_like(u))
    T = torch.cumprod(1.0 - alpha, dim=1)
    Tprev = torch.cat([torch.ones_like(T[:, :1]), T[:, :-1]], dim=1)
    w = Tprev * alpha
    tm = torch.where(mask, t, torch.zeros_like(t))
    N = (w[..., None] * sign[..., None] * nn).sum(1)
    D = (w * tm).sum(1)
    R = (w[..., None] * th["radiance"].T[idx]).sum(1)
    E = (w * th["emissive"][idx]).sum(1)
    P = (w[..., None] * th["albedo"].T[idx]).sum(1)
    A = 1.0 - T[:, -1]
    return N, D, R, E, P, A


def _cosine(Nt, u0, u1):
    h = torch.as_tensor(HELPER, dtype=Nt.dtype)
    m = h[None, :] - (Nt @ h)[:, None] * Nt
    b1 = m / torch.linalg.norm(m, dim=1, keepdim=True)
    b2 = torch.linalg.cross(Nt, b1, dim=1)
    r = torch.sqrt(u0)
    phi = 2.0 * np.pi * u1
    return ((r * torch.cos(phi))[:, None] * b1 + (r * torch.sin(phi))[:, None] * b2
            + torch.sqrt(1.0 - u0)[:, None] * Nt)


def torch_params(scene):
    a = scene.arrays() if hasattr(scene, "arrays") else scene
    th = {k: torch.tensor(np.asarray(a[k], dtype=np.float64), requires_grad=(k in PARAMS))
          for k in PARAMS + ("emissive",)}
    return th


def fixed_forward(th, fwd, cam, prm):
    """Recompute the pixels of `fwd` (render.single_bounce output with
    keep_segments=True) as a differentiable function of th."""
    fr = _frames(th["rot"])
    M = fwd["pixels"].size
    O = torch.from_numpy(fwd["O"])
    W = torch.from_numpy(fwd["W"])
    cam_segs = fwd["cam"]
    idx, mask = _pad([s.hits for s in cam_segs])
    den0 = (W[:, None, :] * fr[2].detach()[idx]).sum(-1)
    sign = torch.where(mask, -torch.sign(den0), torch.zeros_like(den0))
    N, D, R, E, P, A = _segment(th, fr, O, W, idx, mask, sign)
    L = [torch.zeros(3, dtype=torch.float64)] * M
    refl = [i for i in range(M) if fwd["branch"][i] == 2]
    for i in range(M):
        if fwd["branch"][i] == 1:
            L[i] = R[i]
    if refl:
        S = prm.spp
        ri = torch.tensor(refl, dtype=torch.int64)
        Nt = N[ri] / torch.linalg.norm(N[ri], dim=1, keepdim=True)
        Dt = D[ri] / A[ri]
        X = O[ri] + Dt[:, None] * W[ri]
        if prm.detach_bounce:
            X, Nt = X.detach(), Nt.detach()
        rows = np.repeat(np.arange(len(refl)), S)
        samp = np.tile(np.arange(S), len(refl))
        pix = fwd["pixels"][np.array(refl)][rows]
        u0, u1, _, _ = philox.uniforms(pix, samp, 0, prm.camera_id, prm.seed)
        Wd = _cosine(Nt[rows], torch.from_numpy(u0), torch.from_numpy(u1))
        Xr = X[rows]
        sec = [fwd["sec"][refl[r]][s] for r, s in zip(rows, samp)]
        idx2, mask2 = _pad([g.hits for g in sec])
        den1 = (Wd.detach()[:, None, :] * fr[2].detach()[idx2]).sum(-1)
        sign2 = torch.where(mask2, -torch.sign(den1), torch.zeros_like(den1))
        _, _, R1, _, _, _ = _segment(th, fr, Xr, Wd, idx2, mask2, sign2)
        R1m = R1.view(len(refl), S, 3).mean(dim=1)
        for j, i in enumerate(refl):
            L[i] = P[i] * R1m[j]
    return torch.stack(L)


def single_bounce_grad(scene, cam, prm, pixels, dL_dI=None, target=None, fwd=None):
    """Gradient of a loss on the rendered pixels w.r.t. the surfel parameters.

    Loss: sum(dL_dI * I) if dL_dI [M,3] is given (a linear loss), else
    0.5 * sum((I - target)^2) over the pixels. Returns (grads dict of numpy
    arrays in the scene's component-major shapes, image [M,3], fwd)."""
    sc = scene if isinstance(scene, Scene64) else Scene64(scene)
    if fwd is None:
        fwd = single_bounce(sc, cam, prm, pixels=pixels, keep_segments=True)
    th = torch_params(scene)
    L = fixed_forward(th, fwd, cam, prm)
    if dL_dI is not None:
        loss = (L * torch.as_tensor(np.asarray(dL_dI, dtype=np.float64))).sum()
    else:
        loss = 0.5 * ((L - torch.as_tensor(np.asarray(target, dtype=np.float64))) ** 2).sum()
    loss.backward()
    grads = {k: (th[k].grad.numpy().copy() if th[k].grad is not None else np.zeros(th[k].shape)) for k in PARAMS}
    return grads, L.detach().numpy(), fwd


def signature(fwd):
    """The discrete decisions of a single-bounce evaluation."""
    sig = [tuple(fwd["branch"].tolist())]
    for s in fwd["cam"]:
        sig.append(tuple(s.hits.tolist()))
    for row in fwd.get("sec") or []:
        for g in row:
            if g is not None:
                sig.append(tuple(g.hits.tolist()))
    return tuple(sig)
