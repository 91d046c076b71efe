"""Strip-shape autotuner of the fused step.

Times each candidate (strip width, strip height) with the library's
event-timed kernel profile (lbm_profile_step), applies the fastest with
lbm_set_strip_width / lbm_set_tiling and caches the choice in a JSON file
keyed by lattice shapes, instance count and GPU architecture.  Every strip
shape gives bitwise identical results, so tuning never changes the
simulation.  Widths cover strips of 1, 2, 4 and 8 wavefronts, each either
balanced (64 n - 2 columns) or placed at multiples of a multiple of 16
columns (output rows start on 64-byte boundaries); for each width the
uniform plans (chunks of a candidate height) and the balanced plans (1 to 4
workgroups per compute unit, equal shares of rows) are timed.  Beside a fixed
list of heights, each width gets the heights fitted to the GPU: for k = 1..8
the smallest height whose launch has at most k workgroups per compute unit
(a launch just past such a multiple leaves most compute units idle for its
last round of workgroups).  Contexts whose lattice widths are all multiples
of 64 (at most 512) also time the full-row plans (lbm_set_full_rows) at the
same heights.  The two-step kernel (lbm_set_two_step: two time steps per
launch, one-wavefront strips of at most 52 columns) is timed as well, at
widths 52 and 48 (two_step=False leaves it out); a two-step launch counts as
two steps.
"""
from __future__ import annotations

import json
import os

from . import lbm

CANDIDATES = (2, 3, 4, 6, 8, 12, 16, 24, 32, 40, 48, 64)
MIN_HEIGHT = 2  # the smallest strip height lbm_set_tiling accepts
MAX_HEIGHT = 65535  # and the largest
# (output columns per strip): one wavefront per strip, balanced / aligned,
# then strips of 2, 4 and 8 wavefronts, balanced / aligned
WIDTHS = (58, 48, 122, 112, 250, 240, 506, 496)
# strip widths of the two-step kernel (balanced, aligned)
WIDTHS2 = (52, 48)
CACHE = os.environ.get("LBM_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache",
                                                        "lbm_tiling.json"))


def _key(sim, arch: str) -> str:
    shapes = sorted({(p.nx, p.ny) for p in sim.params})
    return f"v5|{arch}|n={sim.n_inst}|" + ",".join(f"{a}x{b}" for a, b in shapes[:8]) + \
        (f"|+{len(shapes) - 8}" if len(shapes) > 8 else "")


def _arch(sim) -> str:
    try:
        return sim.torch.cuda.get_device_properties(sim.device).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


BALANCES = (1, 2, 3, 4)


def apply(sim, width: int, height: int, balance: int = 0, full_rows: int = 0, two_step: int = 0):
    """Strip width, then either uniform chunks of `height` rows or, if balance > 0,
    the balanced plan with `balance` workgroups per compute unit; with
    full_rows, the full-row plan of chunks of `height` rows (width unused);
    with two_step, two steps per launch on that plan."""
    lbm.lbm_set_two_step(sim.ctx, 0)
    if full_rows:
        lbm.lbm_set_tiling(sim.ctx, int(height))
        lbm.lbm_set_full_rows(sim.ctx, 1)
        return
    lbm.lbm_set_strip_width(sim.ctx, int(width))
    if balance > 0:
        lbm.lbm_set_balance(sim.ctx, int(balance))
    else:
        lbm.lbm_set_tiling(sim.ctx, int(height))
    if two_step:
        lbm.lbm_set_two_step(sim.ctx, 1)


def step_ms(sim, nrep: int) -> float:
    """Milliseconds per step of the context's step kernel launched nrep times
    (lbm_profile_step; a two-step launch counts as two steps)."""
    prof = dict(lbm.lbm_profile_step(sim.ctx, nrep))
    if "k_fused_step2" in prof:
        return prof["k_fused_step2"] / 2.0
    return prof["k_fused_step"]


def full_rows_possible(sim) -> bool:
    """Every lattice width a multiple of 64, at most 512 (lbm_set_full_rows)."""
    try:
        lbm.lbm_plan_workgroups(sim.params, 58, 16, 0, 1)
        return True
    except lbm.LBMError:
        return False


def _ncu(sim) -> int:
    try:
        return int(sim.torch.cuda.get_device_properties(sim.device).multi_processor_count)
    except Exception:
        return 256


FIT_KMAX = 8  # workgroups per CU up to which fitted heights are tried


def fitted_heights(sim, width: int, ncu: int, kmax: int = FIT_KMAX, full_rows: int = 0) -> list:
    """For k = 1..kmax the smallest uniform strip height at which the launch has at
    most k * ncu workgroups (the count falls as the height grows); planned on the
    host (lbm_plan_workgroups)."""
    hmin = MIN_HEIGHT
    hmax = min(max(max(p.ny for p in sim.params), hmin), MAX_HEIGHT)

    def count(h):
        return lbm.lbm_plan_workgroups(sim.params, width, h, 0, full_rows)[0]

    out = set()
    for k in range(1, kmax + 1):
        target = k * ncu
        if count(hmax) > target:
            continue
        lo, hi = hmin, hmax
        while lo < hi:
            mid = (lo + hi) // 2
            if count(mid) <= target:
                hi = mid
            else:
                lo = mid + 1
        out.add(lo)
    return sorted(out)


def tune(sim, candidates=CANDIDATES, nrep: int = 30, use_cache: bool = True,
         widths=WIDTHS, balances=BALANCES, two_step: bool = True) -> dict:
    """Pick the fastest strip shape for sim's context; returns the timings."""
    arch = _arch(sim)
    key = _key(sim, arch)
    cache = {}
    if use_cache and os.path.exists(CACHE):
        try:
            with open(CACHE) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache and "two_step" in cache[key]:
        e = cache[key]
        apply(sim, e["width"], e["best"], e["balance"], e["full_rows"], e["two_step"])
        return e
    times = {}
    ncu = _ncu(sim)

    def timed(key, *plan):
        apply(sim, *plan)
        step_ms(sim, 3)  # warm-up
        times[key] = step_ms(sim, nrep)

    for wdt in widths:
        for h in sorted(set(candidates) | set(fitted_heights(sim, wdt, ncu))):
            timed((wdt, h, 0, 0), wdt, h)
        for b in balances:
            timed((wdt, 0, b, 0), wdt, 0, b)
    for wdt in (WIDTHS2 if two_step else ()):
        for h in sorted(set(candidates) | set(fitted_heights(sim, wdt, ncu))):
            timed((wdt, h, 0, 1), wdt, h, 0, 0, 1)
        for b in balances:
            timed((wdt, 0, b, 1), wdt, 0, b, 0, 1)
    if full_rows_possible(sim):  # width 0 marks a full-row plan
        for h in sorted(set(candidates) | set(fitted_heights(sim, 58, ncu, full_rows=1))):
            timed((0, h, 0, 0), 0, h, 0, 1)
    bw, bh, bb, ts = min(times, key=times.get)
    fr = 1 if bw == 0 else 0
    apply(sim, bw, bh, bb, fr, ts)
    entry = {"best": bh, "width": bw, "balance": bb, "full_rows": fr, "two_step": ts,
             "ms": {("2s" if t else "") + (f"fr{h}" if w == 0 else f"{w}x{h}" if b == 0 else f"{w}xbal{b}"): v
                    for (w, h, b, t), v in times.items()}}
    if use_cache:
        cache[key] = entry
        try:
            os.makedirs(os.path.dirname(CACHE), exist_ok=True)
            with open(CACHE, "w") as fh:
                json.dump(cache, fh, indent=1)
        except OSError:
            pass
    return entry


def _main():
    """Print the fused step's time for every strip plan of a sweep (one GPU)."""
    import argparse
    from . import workloads as W
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", default="spinodal",
                    choices=("spinodal", "emulsion", "batched", "adjoint_array"))
    ap.add_argument("--widths", default="240,496,122,58,48")
    ap.add_argument("--heights", default="8:72:2", help="start:stop:step")
    ap.add_argument("--balances", default="1,2,3,4")
    ap.add_argument("--nrep", type=int, default=30)
    ap.add_argument("--two-step", type=int, default=0, help="1: two steps per launch (widths <= 52)")
    a = ap.parse_args()
    ws = W.batched() if a.workload == "batched" else [getattr(W, a.workload)()]
    sim = lbm.Sim([lbm.workload_instance(w) for w in ws])
    h0, h1, hs = (int(v) for v in a.heights.split(":"))
    rows = []
    for wdt in (int(v) for v in a.widths.split(",")):
        plans = [(h, 0) for h in range(h0, h1, hs)] + [(0, int(b)) for b in a.balances.split(",") if b]
        for h, b in plans:
            apply(sim, wdt, h, b, 0, a.two_step)
            step_ms(sim, 3)
            ms = step_ms(sim, a.nrep)
            rows.append((ms, wdt, h, b))
            print(f"width {wdt:4d} {'balance ' + str(b) if b else 'height ' + str(h):>10s}  "
                  f"workgroups {lbm.lbm_get_workgroups(sim.ctx):6d}  "
                  f"{ms:.5f} ms", flush=True)
    rows.sort()
    print("best:", ", ".join(f"{w}x{('bal' + str(b)) if b else h} {ms:.5f} ms" for ms, w, h, b in rows[:8]))
    sim.close()


if __name__ == "__main__":
    _main()
