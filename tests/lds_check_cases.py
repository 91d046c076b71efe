"""Strip, full-row and two-step plans of many shapes run through the checked build of the
library (LDS ring and edge indices counted when out of range); prints the
count.  Run by tests/test_gpu_lds_check.py in a child process with
LBM_HIP_SO pointing at liblbm_hip_check.so."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_1806_06943_amd import lbm  # noqa: E402


def inst(nx, ny, walls, seed):
    r = np.random.default_rng(seed)
    rA = 0.5 + r.uniform(-0.2, 0.2, (ny, nx))
    return dict(nx=nx, ny=ny, rhoA=rA, rhoB=1.0 - rA + 0.03, G_AB=3.0, G1=-7.4, G2=6.4,
                tau=(1.0, 0.7), walls=walls, rho_wall=(0.03, 1.0), g=((1e-5, 0.0), (1e-5, 0.0)))


def main():
    assert os.environ.get("LBM_HIP_SO", "").endswith("liblbm_hip_check.so"), "needs the checked build"
    total = 0
    shapes = [(37, 21, 1), (600, 40, 0), (5, 3, 0), (1, 8, 0), (70, 3, 0), (125, 9, 1), (64, 64, 0)]
    for nx, ny, walls in shapes:
        for cols, h in ((58, 16), (48, 5), (16, 2), (122, 12), (112, 3), (250, 7), (240, 33),
                        (506, 9), (496, 4), (58, -1), (506, -3)):
            sim = lbm.Sim([inst(nx, ny, walls, nx + ny)])
            lbm.lbm_set_strip_width(sim.ctx, cols)
            if h > 0:
                lbm.lbm_set_tiling(sim.ctx, h)
            else:
                lbm.lbm_set_balance(sim.ctx, -h)
            sim.step(3)
            n = lbm.lbm_lds_checks(sim.ctx)
            print(f"strips {cols} x {h} on {nx} x {ny} walls {walls}: {n}", flush=True)
            total += n
            sim.close()
    # full rows: single widths and a mixed context, with a recorded window
    for spec in ([(64, 40, 0)], [(128, 9, 1)], [(192, 5, 0)], [(512, 7, 1)],
                 [(64, 6, 0), (256, 11, 1), (128, 3, 0), (320, 4, 0)]):
        for h in (2, 3, 16):
            sim = lbm.Sim([inst(nx, ny, w, nx * ny) for nx, ny, w in spec])
            lbm.lbm_set_tiling(sim.ctx, h)
            lbm.lbm_set_full_rows(sim.ctx, 1)
            sim.step(3)
            store = sim.torch.empty((3, lbm.lbm_record_floats(sim.ctx, 0)), dtype=sim.torch.float32,
                                    device=sim.device)
            lbm.lbm_record(sim.ctx, 0, 3, store.data_ptr())
            n = lbm.lbm_lds_checks(sim.ctx)
            print(f"full rows {spec} x {h}: {n}", flush=True)
            total += n
            sim.close()
    # two steps per launch: one-wavefront strips of at most 52 columns
    for nx, ny, walls in shapes:
        for cols, h in ((52, 16), (48, 5), (16, 2), (52, -2)):
            sim = lbm.Sim([inst(nx, ny, walls, nx + ny + 1)])
            lbm.lbm_set_strip_width(sim.ctx, cols)
            if h > 0:
                lbm.lbm_set_tiling(sim.ctx, h)
            else:
                lbm.lbm_set_balance(sim.ctx, -h)
            lbm.lbm_set_two_step(sim.ctx, 1)
            sim.step(5)
            n = lbm.lbm_lds_checks(sim.ctx)
            print(f"two steps {cols} x {h} on {nx} x {ny} walls {walls}: {n}", flush=True)
            total += n
            sim.close()
    print(f"LDS_VIOLATIONS {total}", flush=True)


if __name__ == "__main__":
    main()
