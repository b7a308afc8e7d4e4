"""FP64 CPU oracle for 2D-Gaussian surfel tracing, single-bounce rendering
and multi-bounce path tracing.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports, calls or links
this package; only the tests, the smoke check and the benchmark's CPU-baseline
leg do. It shares no code with the HIP library: it reads the float32 scene
arrays made by `scenegen`, upcasts them exactly to float64 and evaluates the
paper's definitions plainly:

* brute force over every surfel for every ray (no acceleration structure);
* a full sort of the accepted hits by the order key;
* compositing over the whole sorted list, stopping at the transmittance
  threshold (Sec. 3.1, Eq. 2-3);
* its own Philox4x32-10 (Salmon et al., SC'11) for every random number.

Modules:
  philox   - counter-based generator from its published definition
  frames   - quaternion frame, pinhole camera, hemisphere frame and
             cosine-weighted direction
  tracer   - ray-surfel intersection, ordering, compositing, decision margins
  render   - 0-bounce, single-bounce (Eq. 5-7) and path-traced (Eq. 9) images
  grad     - the single-bounce map re-expressed in torch.float64 (CPU) with
             every discrete decision fixed, differentiated by autograd
  bake     - light baking: the PQ-encoded L1 loss between 0-bounce and
             path-traced images, its radiance gradient, and the Adam step
  nee      - emitter sampling on emissive surfels combined with cosine
             sampling by multiple importance sampling, for path tracing
  stage0   - the Stage-0 objective (Eq. 4) on the camera segment's Nt, Dt,
             R, E images, with the distance normal, by autograd

Parity status of each function is stated in its module docstring.
"""
from .params import Params  # noqa: F401
