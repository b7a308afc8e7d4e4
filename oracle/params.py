"""Trace and render parameters with the readings this oracle takes.

Defaults (each a reading of a passage that fixes no value):
  tau_E = 0.1        emitter threshold on the composited E (Sec. 3.3, Eq. 5;
                     the paper's own value)
  T_min = 1e-4       transmittance at which compositing stops (Sec. 3.1,
                     "preset threshold", no value given)
  t_min = 1e-3       minimum ray distance of an accepted hit (self-hit guard;
                     not in the paper)
  k_sigma = 3        a surfel's finite extent: accepted iff u^2+v^2 <= k^2
                     (Sec. 3.1 says only "finite spatial extent")
  depth_quantum      order key (floor(t / dq), surfel index); 2^-13 scene
                     units; 0 selects exact (t, index) order (Sec. 3.1
                     "sequentially intersects" is silent on ties)
  max_depth          maximum number of diffuse reflections; a path traces at
                     most max_depth + 1 segments (reading of Eq. 9's bounce
                     count)
  rr_start           Russian roulette applies to reflections that make the
                     depth >= rr_start; 0 disables it (not in the paper)
"""
from dataclasses import dataclass


@dataclass
class Params:
    spp: int = 4
    max_depth: int = 5
    rr_start: int = 3
    tau_E: float = 0.1
    T_min: float = 1e-4
    t_min: float = 1e-3
    k_sigma: float = 3.0
    depth_quantum: float = 2.0 ** -13
    seed: int = 0
    camera_id: int = 0
    jitter: bool = False
    additive: bool = False      # test mode: L_o = L_e + L_r at every hit (first line of Eq. 5)
    detach_bounce: bool = False  # gradient mode: bounce origin and direction held constant
