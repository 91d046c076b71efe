"""Launch the fused step of one workload under a given strip plan, for profilers.

Builds the seeded workload (the same generators as the tests and the
benchmark), applies the strip plan (or tunes it), then times `--launches`
back-to-back launches of the step's kernel on the context's stream with HIP
events (lbm_profile_step) and prints the plan, the workgroup count and the
average time per step (a two-step launch counts as two steps).  Under
``rocprofv3 --pmc ...`` every launch is one dispatch of the counters, so the
per-dispatch averages describe this plan.

    python -m paper_1806_06943_amd.profile_step --workload batched --width 58 --chunk 64
"""
from __future__ import annotations

import argparse

from . import lbm, tune
from . import workloads as W


def build(name: str):
    if name == "batched":
        ws = W.batched()
    elif name == "spinodal":
        ws = [W.spinodal()]
    elif name == "emulsion":
        ws = [W.emulsion()]
    elif name == "adjoint_array":
        ws = [W.adjoint_array()]
    else:
        raise ValueError(name)
    return ws, lbm.Sim([lbm.workload_instance(w) for w in ws])


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", default="batched",
                    choices=("batched", "spinodal", "emulsion", "adjoint_array"))
    ap.add_argument("--width", type=int, default=0, help="strip width (0: tune)")
    ap.add_argument("--chunk", type=int, default=16, help="strip height with --width")
    ap.add_argument("--balance", type=int, default=0, help="workgroups per CU with --width")
    ap.add_argument("--full-rows", action="store_true",
                    help="full-row plan of --chunk rows (lattice widths multiples of 64)")
    ap.add_argument("--two-step", action="store_true",
                    help="two steps per launch (k_fused_step2; --width at most 52)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also launch the library's copy kernel over this many bytes "
                         "(--launches times): the calibration of traffic counters")
    ap.add_argument("--launches", type=int, default=50)
    a = ap.parse_args()
    ws, sim = build(a.workload)
    if a.full_rows:
        tune.apply(sim, 0, a.chunk, 0, 1)
    elif a.width > 0:
        tune.apply(sim, a.width, a.chunk, a.balance, 0, 1 if a.two_step else 0)
    else:
        t = tune.tune(sim, use_cache=False)
        print(f"tuned: width {t['width']} height {t['best']} balance {t['balance']} "
              f"full rows {t['full_rows']} two steps {t['two_step']}", flush=True)
    sim.step(20)
    ms = tune.step_ms(sim, a.launches)
    nodes = sum(w.nx * w.ny for w in ws)
    print(f"{a.workload}: {len(ws)} instances, {nodes} nodes, plan {lbm.lbm_get_strip_width(sim.ctx)} x "
          f"{lbm.lbm_get_tiling(sim.ctx)} balance {lbm.lbm_get_balance(sim.ctx)} "
          f"full rows {lbm.lbm_get_full_rows(sim.ctx)} two steps {lbm.lbm_get_two_step(sim.ctx)}, "
          f"{lbm.lbm_get_workgroups(sim.ctx)} workgroups: {ms:.5f} ms per step, "
          f"{nodes / (ms * 1e-3) / 1e6:.1f} MLUPS, {160.0 * nodes / (ms * 1e-3) / 1e9:.1f} GB/s at "
          f"160 B per lattice update", flush=True)
    if a.copy_bytes > 0:
        t = sim.torch
        src = t.ones(a.copy_bytes // 4, dtype=t.float32, device=sim.device)
        dst = t.empty_like(src)
        e0, e1 = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        for _ in range(a.launches):
            lbm.lbm_copy_probe(sim.ctx, dst.data_ptr(), src.data_ptr(), a.copy_bytes)
        e1.record(sim.stream)
        t.cuda.synchronize()
        ms = e0.elapsed_time(e1) / a.launches
        print(f"copy kernel: {a.copy_bytes} bytes, {ms:.5f} ms per launch, "
              f"{2 * a.copy_bytes / (ms * 1e-3) / 1e9:.1f} GB/s moved", flush=True)
    sim.close()


if __name__ == "__main__":
    main()
