"""Light baking (Sec. 3.4, "Light Baking", Eq. 10), float64.

The per-surfel radiance r is refitted so that the 0-bounce image L_o^0 (the
radiance R composited along the camera ray, Sec. 3.2 "Radiance Loss") of an
edited scene matches path-traced renders of it: min_r L_c(PQ(L_o^0),
PQ(L_o^pt)). Geometry and opacity stay fixed, so the blending weights
w_i = T_{i-1} alpha_i of every camera ray do not depend on r and L_o^0 is
linear in r.

Readings (the paper leaves these open):
* L_c is the L1 term of the usual colour loss, the mean absolute difference
  over pixels and channels; the D-SSIM term is left out.
* PQ is the SMPTE ST 2084 curve applied to Y = max(L, 0) / 10000, i.e. the
  scene's radiance read as cd/m^2. Its derivative, unbounded at Y = 0, is
  taken at max(Y, 2^-24); the derivative of |a - b| at a = b is 0.
* One camera ray per pixel, sample 0 (the pixel centre unless jittered), as
  in the 0-bounce renderer.
* The optimiser is Adam (Kingma and Ba) with bias correction, after which r
  is clamped at 0 (radiance is non-negative).

Functions:
  pq, pq_grad                  the curve and its derivative in L
  bake_loss(L0, Lpt)           loss and dloss/dL0
  zero_bounce_radiance_grad    d<dL, L_o^0>/dr = sum over blended hits of w_i dL
  adam_step                    one projected Adam update

Pinned by tests/test_oracle_bake.py: ST 2084 reference values (PQ of 1, 10,
100, 1000 and 10000 cd/m^2), the PQ derivative and the loss gradient against
central differences, the adjoint identity <dL, L_o^0(r)> = <grad, r> that
linearity gives, a brute-force per-ray weight sum on a tiny scene, and the
closed form of Adam's first step (-lr sign(g)).
"""
import numpy as np

from .render import zero_bounce

PQ_M1 = 2610.0 / 16384.0
PQ_M2 = 2523.0 / 4096.0 * 128.0
PQ_C1 = 3424.0 / 4096.0
PQ_C2 = 2413.0 / 4096.0 * 32.0
PQ_C3 = 2392.0 / 4096.0 * 32.0
PQ_PEAK = 10000.0
PQ_YMIN = 2.0 ** -24


def pq(L):
    """ST 2084 of the linear value L read as cd/m^2 (negative values as 0)."""
    y = np.maximum(np.asarray(L, dtype=np.float64), 0.0) / PQ_PEAK
    ym = y ** PQ_M1
    return ((PQ_C1 + PQ_C2 * ym) / (1.0 + PQ_C3 * ym)) ** PQ_M2


def pq_grad(L):
    """d pq / d L, evaluated at max(Y, 2^-24) (0 where L < 0)."""
    L = np.asarray(L, dtype=np.float64)
    y = np.maximum(L / PQ_PEAK, PQ_YMIN)
    ym = y ** PQ_M1
    num = PQ_C1 + PQ_C2 * ym
    den = 1.0 + PQ_C3 * ym
    base = num / den
    dbase_dym = (PQ_C2 * den - PQ_C3 * num) / (den * den)
    dym_dy = PQ_M1 * y ** (PQ_M1 - 1.0)
    g = PQ_M2 * base ** (PQ_M2 - 1.0) * dbase_dym * dym_dy / PQ_PEAK
    return np.where(L < 0.0, 0.0, g)


def bake_loss(L0, Lpt):
    """Mean |PQ(L0) - PQ(Lpt)| over all values, and its gradient in L0."""
    L0 = np.asarray(L0, dtype=np.float64)
    d = pq(L0) - pq(Lpt)
    n = L0.size
    return float(np.abs(d).sum() / n), np.sign(d) * pq_grad(L0) / n


def zero_bounce_radiance_grad(scene, cam, prm, dL, pixels=None):
    """Gradient of sum(dL * L_o^0) with respect to r, [N, 3]: every blended
    hit i of pixel k adds w_i dL[k] to its surfel's row. dL: [M, 3] for the
    pixels (all pixels if None)."""
    _, segs = zero_bounce(scene, cam, prm, pixels)
    n = scene.N if hasattr(scene, "N") else scene.n
    g = np.zeros((n, 3))
    dL = np.asarray(dL, dtype=np.float64).reshape(len(segs), 3)
    for k, s in enumerate(segs):
        if s.hits.size == 0:
            continue
        T_before = np.concatenate([[1.0], np.cumprod(1.0 - s.alpha)[:-1]])
        w = T_before * s.alpha
        np.add.at(g, s.hits, w[:, None] * dL[k][None, :])
    return g


def adam_step(r, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam update of r with gradient g (step counts from 1), then r is
    clamped at 0. Returns (r, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    r = np.maximum(r - lr * mh / (np.sqrt(vh) + eps), 0.0)
    return r, m, v
