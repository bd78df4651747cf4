"""Write tests/golden/dam_break_2048_ref.npz: the FP64 oracle's state after
1000 steps of the 2048 x 2048 fractal dam break (dx = 2 m, seed 2, 10 m relief,
1 m dam line, 8 m reservoir, open boundaries, psi = 0.4, n = 0.03, Grass bedload
with d50 = 0.5 mm for the critical speed, K = 0.3), started from the
float32-rounded inputs.

Stored: every 16th cell in each direction of h, hu, hv, b (float64), the wet
mask (h > 1e-4 m) of every cell (bit-packed), the water volume, boundary
outflow and model time, and the run's step count.  A second oracle run from
the same inputs with the initial depth multiplied by (1 + 1e-7 N(0,1))
(seeded; float32 rounding level) stores its sampled depth as h_pert: the
spread |h - h_pert| measures how strongly this flow amplifies rounding-level
differences, cell by cell.  Only the oracle and the seeded input generator are
called.  Takes ~20 minutes on 8 cores.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2103_15196_amd import workloads as W  # noqa: E402
from tests.helpers import oracle_case  # noqa: E402

STEPS = 1000
STRIDE = 16
OUT = os.path.join(HERE, "dam_break_2048_ref.npz")


def run(w, label):
    p, inp, s = oracle_case(O, w)
    V0 = O.volumes(p, inp, s)[0]
    t0 = time.time()
    for k in range(STEPS):
        O.step(p, inp, s)
        if (k + 1) % 50 == 0:
            print(f"{label}: step {k + 1}/{STEPS}  t={s.t:.3f}  {time.time() - t0:.0f} s", flush=True)
    return p, inp, s, V0


def main():
    O.build(force=False)
    w = W.dam_break_fractal(n=2048, steps=STEPS).as_float32()
    p, inp, s, V0 = run(w, "reference")
    Vw, Vs = O.volumes(p, inp, s)
    sl = (slice(0, None, STRIDE), slice(0, None, STRIDE))
    wp = W.dam_break_fractal(n=2048, steps=STEPS).as_float32()
    rng = np.random.default_rng(1)
    wp.H = wp.H * (1.0 + 1e-7 * rng.standard_normal(wp.H.shape))
    _, _, sp, _ = run(wp, "perturbed")
    np.savez_compressed(
        OUT, steps=STEPS, stride=STRIDE, t=s.t, V0=V0, Vw=Vw, Vs=Vs, out_w=s.out_w,
        h=s.H[sl], hu=s.qx[sl], hv=s.qy[sl], b=s.b[sl], h_pert=sp.H[sl],
        wet_bits=np.packbits((s.H > 1e-4).reshape(-1)))
    print(f"wrote {OUT} ({os.path.getsize(OUT) / 1e3:.0f} kB)")


if __name__ == "__main__":
    main()
