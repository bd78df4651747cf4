"""Write tests/golden/dam_break_2048_ref.npz: what the FP64 oracle fixes about the
2048 x 2048 fractal dam break (dx = 2 m, seed 2, 10 m relief, 1 m dam line,
8 m reservoir, open boundaries, psi = 0.4, n = 0.03, Grass bedload with
d50 = 0.5 mm for the critical speed, K = 0.3) after 1000 steps, started from
the float32-rounded inputs.

Stored:
* every 16th cell in each direction of h, hu, hv, b (float64), the wet mask
  (h > 1e-4 m) of every cell (bit-packed), the water volume, boundary outflow,
  model time and the Eq. 7 maximum of |v| + c of the final state;
* the problem's sensitivity to float32 rounding: a second run of the same
  algorithm evaluated in float32 arithmetic (oracle.run_f32, the oracle's own
  source compiled with every literal and operation in float32), from the
  same inputs.  For each field, every cell where the two runs differ by more
  than 5e-6 m (h, b) or 5e-6 m times max(|v| + c) (hu, hv) is listed with that
  spread (flat index, float32 spread): the cells where this flow amplifies
  rounding at float32 precision.

Only the oracle (FP64, and its float32 evaluation) and the seeded input
generator are called.  Takes about 20 minutes on 8 cores.
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
LIST_H = 5e-6   # m: spreads listed for h and b above this
OUT = os.path.join(HERE, "dam_break_2048_ref.npz")


def run(w, label, f32=False):
    p, inp, s = oracle_case(O, w)
    V0 = O.volumes(p, inp, s)[0]
    t0 = time.time()
    for k in range(STEPS):
        if f32:
            O.run_f32(p, inp, s, 1)
        else:
            O.step(p, inp, s)
        if (k + 1) % 50 == 0:
            print(f"{label}: step {k + 1}/{STEPS}  t={s.t:.3f}  {time.time() - t0:.0f} s", flush=True)
    return p, inp, s, V0


def sparse(d, thr):
    idx = np.flatnonzero(d.reshape(-1) > thr).astype(np.int32)
    return idx, d.reshape(-1)[idx].astype(np.float32)


def main():
    O.build(force=False)
    w = W.dam_break_fractal(n=2048, steps=STEPS).as_float32()
    p, inp, s, V0 = run(w, "reference")
    Vw, Vs = O.volumes(p, inp, s)
    vs = O.cfl(p, inp, s)["vs"]
    sl = (slice(0, None, STRIDE), slice(0, None, STRIDE))
    _, _, sp, _ = run(w, "float32 evaluation", f32=True)
    lists = {}
    for name, a, b, thr in (("h", s.H, sp.H, LIST_H), ("hu", s.qx, sp.qx, LIST_H * vs),
                            ("hv", s.qy, sp.qy, LIST_H * vs), ("b", s.b, sp.b, LIST_H)):
        idx, val = sparse(np.abs(a - b), thr)
        lists[f"spread_{name}_idx"], lists[f"spread_{name}"] = idx, val
        print(f"{name}: {idx.size} cells spread > {thr:.2e}, max {np.abs(a - b).max():.3e}")
    np.savez_compressed(
        OUT, steps=STEPS, stride=STRIDE, t=s.t, V0=V0, Vw=Vw, Vs=Vs, out_w=s.out_w, vs=vs,
        list_h=LIST_H, h=s.H[sl], hu=s.qx[sl], hv=s.qy[sl], b=s.b[sl],
        wet_bits=np.packbits((s.H > 1e-4).reshape(-1)), **lists)
    print(f"wrote {OUT} ({os.path.getsize(OUT) / 1e3:.0f} kB)")


if __name__ == "__main__":
    main()
