#!/usr/bin/env python3
"""Benchmark: Stokes pair-interactions/s on one MI355X.

Workload: 512 Evans-Fung red blood cells (544 quadrature points each, 278,528
points) placed by random sequential addition in a 120^3 box; single-layer
(Stokeslet) sum from every point to every point of the other cells (same-cell
pairs excluded), densities N(0,1) per component, unit viscosity.  One step =
one full evaluation of that sum (prep, summation and split-reduction kernels).

Reported on one JSON line (stdout):
  value         pair-interactions/s of the headline precision (FP64 by default)
  mixed / fp64  the other precision on the same workload, with its own rate,
                relative L2 error and roofline
  adjoint       single-layer VJP (dL/df and both position gradients, one fused
                pass) time and its ratio to the forward
  roofline      dominant kernel: algorithmic flops (29 per single-layer pair)
                over its measured average duration (HIP events recorded by the
                library on the stream it launches on), against the vector peak
  step_ms       median and minimum of 10 single-step times, taken after the
                timed region (one event pair per step); not part of `value`
  cpu_baseline  the FP64 CPU oracle on a bounded sample of targets (all
                sources), on this host's cores, with the full step's time
                extrapolated from its rate
  configs       the other workload shapes, each in FP64 and mixed precision
                with pairs/s on the pairs evaluated (same-cell pairs not
                counted), a roofline at the stated flops per pair, rel-L2
                against the oracle on a seeded sample, and (128 cells; wall +
                cells) the adjoint and its ratio to the FP64 forward:
                  128 cells (69,632 points), single layer + adjoint;
                  3,840 cells in the vessel, leaf-to-leaf sums;
                  the vessel wall's double layer at 960 cells plus the cells'
                  single layer, superposed, + adjoint.
                --headline-only skips them.

--only checkpoint times the check-point double-layer quadrature on a
vessel-wall ring (every node an on-surface target), --only bie the
30-iteration GMRES solve of the boundary integral equation on an ellipsoid,
--only collision the collision-candidate search of the cells and the wall,
--only fmm the FMM single-layer sum over the cells (and the wall's double layer
at the cells) against the direct sums;
--secondary adds them to the line.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Stokes pair-interactions/s (FP64 vs mixed FP32) at stated rel-L2 error; adjoint/forward"
# MI355X published vector peaks (256 CUs x 2.4 GHz): FP64 128 flop/clk/CU, FP32 256 (packed).
PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3}
# Algorithmic flops per pair interaction (add/sub/mul 1, fma 2, rsqrt 1; Newton
# steps, masks and addressing not counted):
#   single layer, one ordered pair at a time: 29;
#   single layer, each unordered pair once for both points (float64 shared
#   point sets): 10 shared (offset 3, rho^2 5, rsqrt 1, 1/rho^2 1) + 18 per
#   direction (r.q 5, its scale 1, 3 x two fma 12) = 46 per pair = 23 per
#   interaction;
#   double layer: 30.
FLOPS_PER_PAIR_SL = 29
FLOPS_PER_PAIR_SL_SYM = 23
FLOPS_PER_PAIR_DL = 30
KERNEL_NAMES = {"fp64": "sym_main<FwdSL,T=6> (each pair once)", "mixed": "direct_mixed<SL,T=2>",
                "fp64_one_sided": "direct_f64<SL,T=4>"}
PROFILE_TRAFFIC = {"fp64": "sym_main_f64_sl_cfg2_traffic.txt", "mixed": "direct_mixed_sl_cfg2_traffic.txt",
                   "fp64_one_sided": "direct_f64_sl_cfg2_traffic.txt",
                   "p2p_fp64": "p2p_sum_f64_sl_cfg4_traffic.txt", "p2p_mixed": "p2p_sum_mixed_sl_cfg4_traffic.txt"}
PROFILE_SOURCES = {"fp64": ("sym.hip", "direct_dev.hpp", "common.hpp"),
                   "mixed": ("direct.hip", "direct_dev.hpp", "common.hpp"),
                   "fp64_one_sided": ("direct.hip", "direct_dev.hpp", "common.hpp"),
                   "p2p_fp64": ("p2p.hip", "p2p.hpp", "common.hpp"),
                   "p2p_mixed": ("p2p.hip", "p2p.hpp", "common.hpp")}


def path_key(prec, one_sided):
    """The kernel a shared-point single-layer sum of this precision takes."""
    return "fp64_one_sided" if (prec == "fp64" and one_sided) else prec


def flops_sl(prec, one_sided):
    return FLOPS_PER_PAIR_SL_SYM if path_key(prec, one_sided) == "fp64" else FLOPS_PER_PAIR_SL


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(key):
    """Hash of a kernel's sources without comments and whitespace, so that
    counters taken on the same code stay valid across comment edits."""
    h = hashlib.sha256()
    for f in PROFILE_SOURCES[key]:
        with open(os.path.join(ROOT, "paper_1909_11085_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update("".join(text.split()).encode())
    return h.hexdigest()[:16]


def traffic_from_profile(key):
    """HBM bytes per launch from a committed rocprofv3 PMC summary, or None when
    absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", PROFILE_TRAFFIC[key])
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_source_hash(key):
        return None
    return float(m_bytes.group(1))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="headline precision (the other one is reported alongside)")
    ap.add_argument("--only", choices=["fp64", "mixed", "vjp", "p2p", "checkpoint", "bie", "collision", "fmm"],
                    default=None,
                    help="time one path only (for profiler runs); p2p times the leaf-to-leaf "
                         "workload (3,840 cells in the cylinder) in both precisions; checkpoint "
                         "the check-point double-layer quadrature on a vessel-wall ring; bie the "
                         "30-iteration GMRES solve of the boundary integral equation; collision the "
                         "space-time boxes and collision candidates of 3,840 cells and the wall; fmm "
                         "the FMM single-layer sum over those cells against the direct sum")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="target duration of the CPU oracle sample")
    ap.add_argument("--one-sided", action="store_true",
                    help="evaluate every ordered pair separately (pair symmetry off) on the shared point sets")
    ap.add_argument("--headline-only", action="store_true",
                    help="time only the 512-cell workload (skip the 128-cell, leaf-to-leaf and wall + cell "
                         "workloads reported under 'configs')")
    ap.add_argument("--secondary", action="store_true",
                    help="also time the components around the hot path (check points, boundary "
                         "solve, collision candidates, FMM) and report them under 'secondary'")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device-to-device copy (HBM byte-counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU (asked for --gpus {args.gpus}, WORLD_SIZE={world}). "
              "The library has no multi-GPU path: a sharded run would split the targets across "
              "GPUs after one all-gather of the packed sources, with no reduction of outputs.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1909_11085_amd as S
    from paper_1909_11085_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    if args.one_sided:
        S.set_pair_symmetry(False)
    if args.calibrate_copy:
        nbytes = 1 << 30
        a = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": nbytes, "calibrate_copy_bytes_written": nbytes,
                          "launches": 3}), flush=True)
        return
    stream = torch.cuda.current_stream(dev)

    def t(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        S.timing_read()                      # discard warm-up events
        S.timing_enable(True)
        fn()                                 # one more untimed call with the library's timing on
        torch.cuda.synchronize()
        S.timing_read()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for i in range(steps):
            fn()
            ev[i + 1].record(stream)         # step boundaries, for the log
        torch.cuda.synchronize()
        S.timing_enable(False)
        kms, launches = S.timing_read()
        periods = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
        log("  step periods ms: " + " ".join(f"{x:.2f}" for x in periods))
        return ev[0].elapsed_time(ev[steps]) / steps, kms / max(launches, 1), launches

    def per_step(fn, n_steps):
        """Median and minimum of n_steps single-step times (one event pair per
        step), taken after the timed region; they do not enter `value`."""
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_steps)]
        torch.cuda.synchronize()
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        ms = sorted(a.elapsed_time(b) for a, b in ev)
        return {"median": ms[len(ms) // 2], "min": ms[0], "steps": n_steps}

    if args.only == "p2p":
        r = time_p2p(S, W, t, timed, args.steps, args.warmup)
        log(f"p2p: {r}")
        print(json.dumps({"p2p_3840_cells": r}), flush=True)
        return
    if args.only == "fmm":
        r = time_fmm(S, W, t, args.steps, args.warmup)
        log(f"fmm: {r}")
        print(json.dumps({"fmm_3840_cells": r}), flush=True)
        return
    if args.only == "collision":
        r = time_collision(S, W, t, args.steps, args.warmup, oracle=not args.no_cpu_baseline)
        log(f"collision: {r}")
        print(json.dumps({"collision_cells_and_wall": r}), flush=True)
        return
    if args.only == "bie":
        r = time_bie(S, W, t, args.steps, args.warmup)
        log(f"bie: {r}")
        print(json.dumps({"bie_solve_ellipsoid": r}), flush=True)
        return
    if args.only == "checkpoint":
        r = time_checkpoint(S, W, t, timed, args.steps, args.warmup, oracle=not args.no_cpu_baseline)
        log(f"checkpoint: {r}")
        print(json.dumps({"checkpoint_wall_ring": r}), flush=True)
        return

    t0 = time.time()
    cfg = W.make_config(2)
    cells, f = cfg["cells"], cfg["f"]
    n = cells.n
    pairs = W.pair_count_direct(cells.group, cells.group, True)
    log(f"workload: {cells.meta['n_cells']} cells, {n} points, {pairs} pairs/step "
        f"(generated in {time.time() - t0:.1f}s)")

    pos, ft, wt, grp, gh = t(cells.pos), t(f), t(cells.weight), t(cells.group), t(cells.group_h)
    out = torch.empty((3, n), dtype=torch.float64, device=dev)

    def fwd(precision):
        S.sl(pos, ft, wt, pos, src_group=grp, trg_group=grp, precision=precision, group_h=gh,
             near_frac=0.5, out=out)

    results = {}
    outputs = {}
    precisions = [args.precision, "mixed" if args.precision == "fp64" else "fp64"]
    if args.only in ("fp64", "mixed"):
        precisions = [args.only]
    if args.only != "vjp":
        for prec in precisions:
            ms, kms, launches = timed(lambda: fwd(prec), args.steps, args.warmup)
            outputs[prec] = out.cpu().numpy()
            rate = pairs / (ms * 1e-3)
            fl = flops_sl(prec, args.one_sided)
            achieved = pairs * fl / (kms * 1e-3) / 1e12
            results[prec] = dict(ms_per_step=ms, value=rate, kernel_ms=kms, launches=launches,
                                 achieved=achieved, step_ms=per_step(lambda: fwd(prec), 10))
            log(f"{prec}: {ms:.3f} ms/step, {rate:.4e} pairs/s, main kernel {kms:.3f} ms "
                f"({achieved:.2f} TFLOP/s at {fl} flop/pair)")

    # adjoint of L = 0.5 |u - u_ref|^2 at a fixed cotangent g (FP64, fused shared-point pass)
    adjoint = None
    if args.only in (None, "vjp") and hasattr(S, "sl_vjp"):
        g = t(np.random.default_rng(7).standard_normal((3, n)))
        gf = torch.empty_like(ft)
        gs = torch.empty_like(pos)
        gx = torch.empty_like(pos)

        def bwd():
            S.sl_vjp(pos, ft, wt, pos, g, src_group=grp, trg_group=grp,
                         grad_f=gf, grad_src=gs, grad_trg=gs)

        ms, kms, launches = timed(bwd, max(1, args.steps // 2), 1)
        fwd_ms = results.get("fp64", {}).get("ms_per_step")
        adjoint = dict(ms_per_step=ms, kernel_ms=kms, outputs=["dL/df", "dL/dsrc", "dL/dtrg"],
                       precision="fp64",
                       ratio_to_forward=(ms / fwd_ms) if fwd_ms else None)
        log(f"adjoint: {ms:.3f} ms/step" + (f", {ms / fwd_ms:.2f}x forward" if fwd_ms else ""))

    # CPU oracle on a bounded sample of targets; its outputs also give the error
    cpu = None
    rel = {}
    if not args.no_cpu_baseline and args.only is None:
        from oracle import oracle as O

        rng = np.random.default_rng(2025)
        pilot = W.subset(rng, n, 256)
        tp = time.time()
        O.sl(cells.pos, f, cells.weight, cells.pos[:, pilot], src_group=cells.group,
             trg_group=cells.group[pilot], exclude_same_group=True)
        rate_pilot = 256 * n / (time.time() - tp)
        m = int(min(n, max(512, args.cpu_seconds * rate_pilot / n)))
        idx = W.subset(rng, n, m)
        tc = time.time()
        ref = O.sl(cells.pos, f, cells.weight, cells.pos[:, idx], src_group=cells.group,
                   trg_group=cells.group[idx], exclude_same_group=True)
        dt = time.time() - tc
        cpu_pairs = int(W.pair_count_direct(cells.group, cells.group[idx], True))
        cpu = dict(value=cpu_pairs / dt, unit="pair-interactions/s", cores=O.num_threads(),
                   kind="oracle",
                   sample=f"{m} seeded targets x all {n} sources ({cpu_pairs} pairs, FP64, "
                          f"{dt:.1f} s, compensated sums)",
                   extrapolated_full_step_s=pairs / (cpu_pairs / dt))
        log(f"cpu oracle: {cpu['value']:.4e} pairs/s on {cpu['cores']} threads ({dt:.1f}s)")
        for prec, u in outputs.items():
            rel[prec] = float(np.linalg.norm(u[:, idx] - ref) / np.linalg.norm(ref))
            log(f"{prec}: rel-L2 vs oracle on {m} targets = {rel[prec]:.3e}")

    head = args.precision if args.precision in results else (args.only or args.precision)
    hr = results.get(head)

    def roofline(prec):
        r = results[prec]
        key = path_key(prec, args.one_sided)
        return {"bound": "alu", "achieved": round(r["achieved"], 3), "peak": PEAK_TFLOPS[prec],
                "unit": "TFLOP/s", "frac": round(r["achieved"] / PEAK_TFLOPS[prec], 4),
                "traffic": traffic_from_profile(key), "kernel": KERNEL_NAMES[key],
                "flops_per_pair": flops_sl(prec, args.one_sided), "pairs_per_launch": pairs,
                "kernel_ms": round(r["kernel_ms"], 4)}

    line = {
        "metric": METRIC,
        "value": hr["value"] if hr else None,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hr["ms_per_step"] if hr else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "512 Evans-Fung RBCs (p=16, 544 pts each, 278,528 points) in a 120^3 "
                               "box; single-layer Stokeslet direct sum, all points to all points, "
                               "same-cell pairs excluded",
                   "precision": head, "n_points": n, "pairs_per_step": pairs, "mu": 1.0},
        "rel_l2": rel.get(head),
        "step_ms": hr["step_ms"] if hr else None,
    }
    if hr:
        line["roofline"] = roofline(head)
    other = [p for p in results if p != head]
    for p in other:
        line[p] = {"value": results[p]["value"], "ms_per_step": results[p]["ms_per_step"],
                   "step_ms": results[p]["step_ms"], "rel_l2": rel.get(p), "roofline": roofline(p),
                   "speedup_vs_" + head: results[head]["ms_per_step"] / results[p]["ms_per_step"]
                   if hr else None}
    if adjoint:
        line["adjoint"] = adjoint
    line["cpu_baseline"] = cpu
    if not args.headline_only and args.only is None:
        oracle = not args.no_cpu_baseline
        line["configs"] = {}
        for name, fn, st in (("cfg3_128_cells", bench_cfg3, 10), ("cfg4_p2p_3840_cells", bench_cfg4, 10),
                             ("cfg5_wall_and_960_cells", bench_cfg5, 3)):
            tc = time.time()
            line["configs"][name] = fn(S, W, t, timed, st, oracle, args.one_sided)
            log(f"{name} ({time.time() - tc:.1f}s): " + json.dumps(line["configs"][name]))
    if args.secondary:
        line["secondary"] = secondary(S, W, t, timed, log)
    print(json.dumps(line), flush=True)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _roofline(prec, flops, kernel_ms, kernel):
    """Algorithmic flops of one step over its summation kernels' time."""
    ach = flops / (kernel_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
            "frac": round(ach / PEAK_TFLOPS[prec], 4), "kernel": kernel, "kernel_ms": round(kernel_ms, 4)}


def bench_cfg3(S, W, t, timed, steps, oracle, one_sided=False):
    """128 cells (69,632 points): single layer forward in both precisions and
    the fused adjoint of L = 0.5 |u - u_ref|^2 (dL/df and the total dL/dx)."""
    import torch

    cfg = W.make_config(3)
    c, f, u_ref = cfg["cells"], cfg["f"], cfg["u_ref"]
    n = c.n
    pos, ft, wt, grp, gh = t(c.pos), t(f), t(c.weight), t(c.group), t(c.group_h)
    pairs = W.pair_count_direct(c.group, c.group, True)
    r = {"workload": "128 Evans-Fung RBCs (69,632 points) in a 75.6^3 box; single-layer sum all points to "
                     "all points, same-cell pairs excluded; adjoint of L = 0.5 |u - u_ref|^2",
         "pairs": pairs}
    outs = {}
    for prec in ("fp64", "mixed"):
        u = torch.empty((3, n), dtype=torch.float64, device=pos.device)
        ms, kms, la = timed(lambda: S.sl(pos, ft, wt, pos, src_group=grp, trg_group=grp, precision=prec,
                                         group_h=gh, out=u), steps, 2)
        outs[prec] = u.cpu().numpy()
        km = kms * la / steps
        key = path_key(prec, one_sided)
        r[prec] = {"ms_per_step": ms, "pairs_per_s": pairs / (ms * 1e-3),
                   "roofline": dict(_roofline(prec, pairs * flops_sl(prec, one_sided), km, KERNEL_NAMES[key]),
                                    flops_per_pair=flops_sl(prec, one_sided))}
    r["mixed_speedup_vs_fp64"] = r["fp64"]["ms_per_step"] / r["mixed"]["ms_per_step"]
    g = t(outs["fp64"]) - t(u_ref)
    gf, gx = torch.empty_like(ft), torch.empty_like(pos)
    ms, _, _ = timed(lambda: S.sl_vjp(pos, ft, wt, pos, g, src_group=grp, trg_group=grp, grad_f=gf,
                                      grad_src=gx, grad_trg=gx), steps, 1)
    r["adjoint"] = {"ms_per_step": ms, "outputs": ["dL/df", "dL/dx (total)"], "precision": "fp64",
                    "ratio_to_fp64_forward": ms / r["fp64"]["ms_per_step"]}
    if oracle:
        from oracle import oracle as O

        idx = W.subset(np.random.default_rng(3003), n, 512)
        ref = O.sl(c.pos, f, c.weight, c.pos[:, idx], src_group=c.group, trg_group=c.group[idx],
                   exclude_same_group=True)
        for prec in ("fp64", "mixed"):
            r[prec]["rel_l2"] = _rel(outs[prec][:, idx], ref)
        gh_ = g.cpu().numpy()
        _, _, rt = O.sl_vjp(c.pos, f, c.weight, c.pos[:, idx], gh_[:, idx], src_group=c.group,
                            trg_group=c.group[idx], exclude_same_group=True, want=("trg",))
        rf, rs, _ = O.sl_vjp(c.pos[:, idx], f[:, idx], c.weight[idx], c.pos, gh_, src_group=c.group[idx],
                             trg_group=c.group, exclude_same_group=True, want=("f", "src"))
        r["adjoint"]["rel_l2"] = {"dL/df": _rel(gf.cpu().numpy()[:, idx], rf),
                                  "dL/dx": _rel(gx.cpu().numpy()[:, idx], rs + rt)}
        r["oracle_sample"] = "512 seeded points x all sources"
    return r


def bench_cfg4(S, W, t, timed, steps, oracle, one_sided=False):
    """3,840 cells (2,088,960 points) in the cylinder, octree leaves of <= 256
    points, lists of 27..60 leaves: the leaf-to-leaf sum in one launch."""
    cfg = W.make_config(4)
    c, tree, f = cfg["cells"], cfg["tree"], cfg["f"]
    ofs, ul = cfg["ulist_ofs"], cfg["ulist"]
    plan = S.P2PPlan(tree.leaf_ofs, tree.leaf_ofs, ofs, ul, c.n, c.n)
    pos, ft, wt, grp, gh = t(c.pos), t(f), t(c.weight), t(c.group), t(c.group_h)
    pairs = W.pair_count_p2p(tree.leaf_ofs, ofs, ul, c.group, True)
    r = {"workload": "3,840 Evans-Fung RBCs (2,088,960 points) in a cylinder (radius 50, length 400); "
                     "octree leaves of <= 256 points, each leaf summing over its 27..60 nearest leaves; "
                     "single layer, same-cell pairs excluded",
         "pairs": pairs, "listed_pairs": plan.pairs(), "leaves": len(tree.leaf_ofs) - 1}
    # the leaf layout as device arrays, passed per call (the items are built,
    # checked and sorted on the device inside the timed step)
    lay = (t(tree.leaf_ofs.astype(np.int64)), t(tree.leaf_ofs.astype(np.int64)), t(ofs.astype(np.int64)),
           t(ul.astype(np.int32)))
    r["layout"] = "device leaf arrays per call (stokes_p2p_leaf_eval)"
    outs = {}
    for prec in ("fp64", "mixed"):
        ms, kms, la = timed(lambda: S.p2p_leaf(lay, pos, ft, wt, pos, src_group=grp, trg_group=grp,
                                               precision=prec, group_h=gh), steps, 2)
        outs[prec] = S.p2p_leaf(lay, pos, ft, wt, pos, src_group=grp, trg_group=grp, precision=prec,
                                group_h=gh).cpu().numpy()
        km = kms * la / steps
        ms_plan, _, _ = timed(lambda: S.p2p_leaf(plan, pos, ft, wt, pos, src_group=grp, trg_group=grp,
                                                 precision=prec, group_h=gh), steps, 2)
        r[prec] = {"ms_per_step": ms, "pairs_per_s": pairs / (ms * 1e-3), "plan_ms_per_step": ms_plan,
                   "roofline": dict(_roofline(prec, pairs * FLOPS_PER_PAIR_SL, km,
                                              "p2p_sum<SL,%s>" % ("FP64" if prec == "fp64" else "mixed")),
                                    flops_per_pair=FLOPS_PER_PAIR_SL, traffic=traffic_from_profile("p2p_" + prec))}
    r["mixed_speedup_vs_fp64"] = r["fp64"]["ms_per_step"] / r["mixed"]["ms_per_step"]
    if oracle:
        from oracle import oracle as O

        leaves = np.random.default_rng(4004).choice(len(tree.leaf_ofs) - 1, size=48, replace=False)
        tt, ref = [], []
        for L in leaves:
            ti = np.arange(tree.leaf_ofs[L], tree.leaf_ofs[L + 1])
            si = np.concatenate([np.arange(tree.leaf_ofs[k], tree.leaf_ofs[k + 1]) for k in ul[ofs[L]:ofs[L + 1]]])
            ref.append(O.sl(c.pos[:, si], f[:, si], c.weight[si], c.pos[:, ti], src_group=c.group[si],
                            trg_group=c.group[ti], exclude_same_group=True))
            tt.append(ti)
        tt, ref = np.concatenate(tt), np.concatenate(ref, 1)
        for prec in ("fp64", "mixed"):
            r[prec]["rel_l2"] = _rel(outs[prec][:, tt], ref)
        r["oracle_sample"] = "48 seeded leaves (%d targets) x their listed sources" % len(tt)
    return r


def bench_cfg5(S, W, t, timed, steps, oracle, one_sided=False):
    """Wall + cells: the wall's double layer (1,048,576 nodes) at the 522,240
    points of 960 cells plus the cells' single layer (same-cell rule), added
    into one velocity; then the adjoint of L = 0.5 |u - u_ref|^2 with respect
    to the wall density, the cell densities and the cell positions."""
    import torch

    cfg = W.make_config(5)
    wall, c = cfg["wall"], cfg["cells"]
    wp, wphi, ww, wn, wg, wh = (t(wall.pos), t(cfg["phi"]), t(wall.weight), t(wall.normal),
                                t(wall.group), t(wall.group_h))
    cp, cf, cw, cg, ch = t(c.pos), t(cfg["f"]), t(c.weight), t(c.group), t(c.group_h)
    dl_pairs = wall.n * c.n
    sl_pairs = W.pair_count_direct(c.group, c.group, True)
    r = {"workload": "vessel wall (cylinder radius 50, length 400, 4,096 patches of 16 x 16 nodes: 1,048,576 "
                     "points) double layer at the 522,240 points of 960 Evans-Fung RBCs, plus the cells' "
                     "single layer (same-cell pairs excluded), superposed; adjoint of L = 0.5 |u - u_ref|^2",
         "dl_pairs": dl_pairs, "sl_pairs": sl_pairs, "pairs": dl_pairs + sl_pairs}
    outs = {}
    for prec in ("fp64", "mixed"):
        u = torch.empty((3, c.n), dtype=torch.float64, device=cp.device)

        def both():
            S.dl(wp, wphi, ww, wn, cp, src_group=wg, precision=prec, group_h=wh, exclude_same_group=False,
                 out=u)
            S.sl(cp, cf, cw, cp, src_group=cg, trg_group=cg, precision=prec, group_h=ch, out=u,
                 accumulate=True)

        ms, kms, la = timed(both, steps, 1)
        outs[prec] = u.cpu().numpy()
        km = kms * la / steps
        flops = dl_pairs * FLOPS_PER_PAIR_DL + sl_pairs * flops_sl(prec, one_sided)
        r[prec] = {"ms_per_step": ms, "pairs_per_s": (dl_pairs + sl_pairs) / (ms * 1e-3),
                   "roofline": dict(_roofline(prec, flops, km, "direct_%s<DL> + %s" % (
                       prec, KERNEL_NAMES[path_key(prec, one_sided)])),
                       flops_per_pair_dl=FLOPS_PER_PAIR_DL, flops_per_pair_sl=flops_sl(prec, one_sided))}
    r["mixed_speedup_vs_fp64"] = r["fp64"]["ms_per_step"] / r["mixed"]["ms_per_step"]
    g = t(outs["fp64"]) - t(cfg["u_ref"])
    gphi, gfc, gx = torch.empty_like(wphi), torch.zeros_like(cf), torch.empty_like(cp)

    def adj():
        S.dl_vjp(wp, wphi, ww, wn, cp, g, grad_phi=gphi, grad_trg=gx)
        S.sl_vjp(cp, cf, cw, cp, g, src_group=cg, trg_group=cg, grad_f=gfc, grad_src=gx, grad_trg=gx,
                 accumulate=True)

    gfc.zero_()
    ms, _, _ = timed(adj, max(1, steps // 2), 1)
    r["adjoint"] = {"ms_per_step": ms, "outputs": ["dL/dphi (wall)", "dL/df (cells)", "dL/dx (cells, total)"],
                    "precision": "fp64", "ratio_to_fp64_forward": ms / r["fp64"]["ms_per_step"]}
    if oracle:
        from oracle import oracle as O

        it = W.subset(np.random.default_rng(5005), c.n, 256)
        ref = O.dl(wall.pos, cfg["phi"], wall.weight, wall.normal, c.pos[:, it])
        ref += O.sl(c.pos, cfg["f"], c.weight, c.pos[:, it], src_group=c.group, trg_group=c.group[it],
                    exclude_same_group=True)
        for prec in ("fp64", "mixed"):
            r[prec]["rel_l2"] = _rel(outs[prec][:, it], ref)
        # one adjoint call more, from zero (the timed calls accumulated into dL/df)
        gfc.zero_()
        adj()
        gh_ = g.cpu().numpy()
        iw = W.subset(np.random.default_rng(5006), wall.n, 256)
        rp = O.dl_vjp(wall.pos[:, iw], cfg["phi"][:, iw], wall.weight[iw], wall.normal[:, iw], c.pos, gh_,
                      want=("phi",))[0]
        rx = O.dl_vjp(wall.pos, cfg["phi"], wall.weight, wall.normal, c.pos[:, it], gh_[:, it], want=("trg",))[2]
        rx += O.sl_vjp(c.pos, cfg["f"], c.weight, c.pos[:, it], gh_[:, it], src_group=c.group,
                       trg_group=c.group[it], exclude_same_group=True, want=("trg",))[2]
        rf, rs, _ = O.sl_vjp(c.pos[:, it], cfg["f"][:, it], c.weight[it], c.pos, gh_, src_group=c.group[it],
                             trg_group=c.group, exclude_same_group=True, want=("f", "src"))
        r["adjoint"]["rel_l2"] = {"dL/dphi": _rel(gphi.cpu().numpy()[:, iw], rp),
                                  "dL/df": _rel(gfc.cpu().numpy()[:, it], rf),
                                  "dL/dx": _rel(gx.cpu().numpy()[:, it], rx + rs)}
        r["oracle_sample"] = "256 seeded cell points (and 256 wall nodes for dL/dphi) x all sources"
    return r


def time_p2p(S, W, t, timed, steps, warmup):
    """Leaf-to-leaf sums of 3,840 cells in the cylinder (lists of 27..60 leaves), both precisions;
    rates on the pairs evaluated (same-cell pairs of the lists not counted)."""
    cfg = W.make_config(4)
    c, tree, f = cfg["cells"], cfg["tree"], cfg["f"]
    plan = S.P2PPlan(tree.leaf_ofs, tree.leaf_ofs, cfg["ulist_ofs"], cfg["ulist"], c.n, c.n)
    pos, ft, wt, grp, gh = t(c.pos), t(f), t(c.weight), t(c.group), t(c.group_h)
    pairs = W.pair_count_p2p(tree.leaf_ofs, cfg["ulist_ofs"], cfg["ulist"], c.group, True)
    lay = (t(tree.leaf_ofs.astype(np.int64)), t(tree.leaf_ofs.astype(np.int64)),
           t(cfg["ulist_ofs"].astype(np.int64)), t(cfg["ulist"].astype(np.int32)))
    r = {"pairs": pairs, "listed_pairs": plan.pairs(), "leaves": len(tree.leaf_ofs) - 1,
         "layout": "device leaf arrays per call"}
    for prec in ("mixed", "fp64"):
        ms, kms, _ = timed(lambda: S.p2p_leaf(lay, pos, ft, wt, pos, src_group=grp, trg_group=grp,
                                              precision=prec, group_h=gh), steps, warmup)
        r[f"{prec}_ms"] = ms
        r[f"{prec}_kernel_ms"] = kms
        r[f"{prec}_pairs_per_s"] = pairs / (ms * 1e-3)
    return r


def time_checkpoint(S, W, t, timed, steps, warmup, oracle=True):
    """Check-point double-layer quadrature (Sec. 3.1) with every node of a
    vessel-wall ring as an on-surface target: 64 x 4 patches of 16 x 16
    Gauss-Legendre nodes (the 1M-node wall's patch shape), eta = 1 (4
    sub-squares), p = 8, R = r = 0.15 L.  One step = upsampling, check points,
    the double-layer sum over the fine nodes at every check point, and the
    extrapolation.  The timed kernel is that sum (30 flop per pair)."""
    wall = W.cylinder_wall(radius=50.0, length=25.0, n_theta=64, n_z=4, q=16)
    phi = np.random.default_rng(11).standard_normal((3, wall.n))
    tq, wq = wall.meta["nodes_1d"], wall.meta["weights_1d"]
    eta, p, R = 1, 8, 0.15
    n_fine = wall.n * 4 ** eta
    n_check = wall.n * (p + 1)
    pairs = n_fine * n_check
    X, F = t(wall.pos), t(phi)
    r = {"targets": wall.n, "fine_sources": n_fine, "check_points": n_check, "pairs": pairs,
         "eta": eta, "p": p, "R_over_L": R, "r_over_L": R, "kernel": "direct_f64<DL,T=4> / direct_mixed<DL>",
         "flops_per_pair": FLOPS_PER_PAIR_DL}
    outs = {}
    for prec in ("fp64", "mixed"):
        ms, kms, _ = timed(lambda: outs.__setitem__(prec, S.dl_checkpoint(X, F, tq, wq, eta=eta, p=p, R_frac=R,
                                                                           r_frac=R, precision=prec)),
                           steps, warmup)
        ach = pairs * FLOPS_PER_PAIR_DL / (kms * 1e-3) / 1e12
        r[f"{prec}_ms"] = ms
        r[f"{prec}_sum_kernel_ms"] = kms
        r[f"{prec}_targets_per_s"] = wall.n / (ms * 1e-3)
        r[f"{prec}_pairs_per_s"] = pairs / (ms * 1e-3)
        r[f"{prec}_sum_tflops"] = ach
        r[f"{prec}_sum_frac_of_peak"] = ach / PEAK_TFLOPS[prec]
        r[f"{prec}_outside_sum_ms"] = ms - kms
    if oracle:                           # CPU baseline leg: the oracle on a sample; it also gives the error
        from oracle import hedgehog as H
        from oracle import oracle as O

        pick = W.subset(np.random.default_rng(12), wall.n, 48)
        pt, u, v, d = H.on_surface_targets(wall.meta["n_patches"], tq)
        tc = time.time()
        ref = H.singular_dl(wall.pos, phi, tq, wq, eta, p, R, R, pt[pick], u[pick], v[pick], d[pick])
        dt = time.time() - tc
        r["cpu_baseline"] = {"value": len(pick) / dt, "unit": "targets/s", "cores": O.num_threads(),
                             "kind": "oracle",
                             "sample": f"{len(pick)} seeded targets, upsampling of all patches included, "
                                       f"{dt:.1f} s"}
        for prec, u_gpu in outs.items():
            got = u_gpu.cpu().numpy()[:, pick]
            r[f"{prec}_rel_l2_sample"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    return r


def time_bie(S, W, t, steps, warmup):
    """GMRES solve of the boundary integral equation (eq. int_eq_disc), capped
    at 30 iterations as in the paper's scaling runs, on an ellipsoid (semi-axes
    1, 0.9, 0.8) of 6 x 3 x 3 patches of 16 x 16 nodes (13,824 nodes), eta = 2,
    p = 8, R = r = 0.15 L, boundary data of a point force outside.  One step =
    one solve (30 matrix-vector products, each a check-point quadrature over
    221,184 fine nodes at 124,416 check points, plus the Arnoldi vector work)."""
    import torch

    s = W.cube_sphere(1.0, m=3, q=16, axes=(1.0, 0.9, 0.8))
    tq, wq = s.meta["nodes_1d"], s.meta["weights_1d"]
    x0, F = np.array([[1.7], [0.6], [-0.5]]), np.array([[0.3], [-1.0], [0.5]])

    def point_force(x):                   # its velocity, by the library's single-layer sum
        return S.sl(t(x0), t(F), t(np.ones(1)), x)

    X = t(s.pos)
    g = point_force(X)
    its_cap, eta, p = 30, 2, 8
    n_fine, n_check = s.n * 4 ** eta, s.n * (p + 1)
    pairs = n_fine * n_check
    for _ in range(warmup):
        S.bie_solve(X, g, tq, wq, eta=eta, p=p, max_iter=its_cap, rtol=0.0)
    torch.cuda.synchronize()
    S.timing_read()
    S.timing_enable(True)
    t0 = time.time()
    for _ in range(steps):
        phi, its, hist = S.bie_solve(X, g, tq, wq, eta=eta, p=p, max_iter=its_cap, rtol=0.0)
    torch.cuda.synchronize()
    ms = (time.time() - t0) * 1e3 / steps
    S.timing_enable(False)
    kms, launches = S.timing_read()
    sum_ms = kms / max(launches, 1)
    rng = np.random.default_rng(41)
    xin = rng.standard_normal((3, 64))
    xin *= 0.5 * rng.uniform(0, 1, 64) ** (1 / 3) / np.linalg.norm(xin, axis=0)
    u = S.dl(X, phi, t(s.weight), t(s.normal), t(xin)).cpu().numpy()
    ue = point_force(t(xin)).cpu().numpy()
    return {"nodes": s.n, "fine_sources": n_fine, "check_points": n_check, "iterations": its,
            "pairs_per_matvec": pairs, "solve_ms": ms, "ms_per_iteration": ms / its,
            "dl_sum_kernel_ms": sum_ms, "dl_sum_share": sum_ms * its / ms,
            "dl_sum_tflops": pairs * FLOPS_PER_PAIR_DL / (sum_ms * 1e-3) / 1e12,
            "final_residual": float(hist[-1]),
            "interior_rel_error": float(np.abs(u - ue).max() / np.abs(ue).max()),
            "precision": "fp64", "timing": "host clock around the blocking solve"}


def time_collision(S, W, t, steps, warmup, oracle=True):
    """Collision candidates (Sec. 4): space-time boxes of the 3,840 cells of
    the cylinder workload over one time step (rigid random shifts of up to 0.5
    and turns of up to 0.05 rad per cell) and boxes of the 4,096 static wall
    patches, then the pairs of boxes sharing a cell of the grid whose spacing
    is the mean box diagonal.  One step = both box kernels and one candidate
    search.  The box kernels read every point at both time levels once."""
    import torch
    from types import SimpleNamespace

    cfg = W.make_config(4)
    cells = cfg["cells"]
    order = np.argsort(cells.group, kind="stable")
    pos = np.ascontiguousarray(cells.pos[:, order])
    grp = cells.group[order]
    x1 = W.cells_after_step(np.random.default_rng(66), SimpleNamespace(pos=pos, group=grp))
    ofs = W.group_offsets(grp)
    wall = W.cylinder_wall()
    wofs = np.arange(0, wall.n + 1, wall.meta["points_per_patch"], dtype=np.int64)
    P0, P1, O, WP, WO = t(pos), t(x1), t(ofs), t(wall.pos), t(wofs)
    nc, nw = len(ofs) - 1, len(wofs) - 1
    lo = torch.empty((3, nc + nw), dtype=torch.float64, device=P0.device)
    hi = torch.empty_like(lo)
    box_bytes = (2 * pos.shape[1] + wall.n) * 24 + (len(ofs) + len(wofs)) * 8 + 2 * (nc + nw) * 48

    def boxes():
        a, b = S.space_time_boxes(O, P0, P1)
        c, d = S.space_time_boxes(WO, WP)
        lo[:, :nc], lo[:, nc:], hi[:, :nc], hi[:, nc:] = a, c, b, d

    boxes()
    H = float((hi - lo).norm(dim=0).mean())
    pairs = S.collision_candidates(lo, hi, H)
    cap = pairs.shape[1]
    for _ in range(warmup):
        boxes()
        S.collision_candidates(lo, hi, H, capacity=cap)
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    box_ms = search_ms = 0.0
    t0 = time.time()
    for _ in range(steps):
        e0.record()
        boxes()
        e1.record()
        pairs = S.collision_candidates(lo, hi, H, capacity=cap)
        e2.record()
        torch.cuda.synchronize()
        box_ms += e0.elapsed_time(e1)
        search_ms += e1.elapsed_time(e2)
    ms = (time.time() - t0) * 1e3 / steps
    r = {"meshes": nc + nw, "cells": nc, "wall_patches": nw, "points_read": 2 * pos.shape[1] + wall.n,
         "cell_size": H, "candidate_pairs": int(pairs.shape[1]), "step_ms": ms, "boxes_ms": box_ms / steps,
         "boxes_GBps": box_bytes / (box_ms / steps * 1e-3) / 1e9, "boxes_bytes": box_bytes,
         "search_ms": search_ms / steps, "note": "boxes_ms includes the slicing copies into one box array"}
    if oracle:                           # CPU baseline leg: the oracle's search on the same boxes
        from oracle import spatial as SP

        hlo, hhi = lo.cpu().numpy(), hi.cpu().numpy()
        tc = time.time()
        ref = SP.collision_candidates(hlo, hhi, H)
        dt = time.time() - tc
        r["cpu_baseline"] = {"value": 1e3 * dt, "unit": "ms per search", "cores": 1, "kind": "oracle",
                             "sample": f"the whole search over {nc + nw} boxes, brute force over pairs"}
        got = {tuple(p) for p in pairs.cpu().numpy().T.tolist()}
        r["matches_oracle"] = got == {tuple(p) for p in ref.tolist()}
    return r


def time_fmm(S, W, t, steps, warmup):
    """The single-layer sum over all 2,088,960 points of the 3,840 cells in the
    vessel (every point a source and a target, no pair rule) by the FMM on a
    uniform octree (depth 6 at surface orders 4 and 6, depth 5 at orders 8 and
    10, where the larger far-field operators favour fewer levels), against the
    direct sum (timed once; its 4.4e12 pairs are the O(N^2) baseline) on a
    seeded sample of 2,000 targets for the error.  Each order also runs with
    precision="mixed" (float32 near-field pairs).  Then the wall's double
    layer at the cells' points (cfg5) at orders 6 and 10.  Plan creation (the
    operators; about 26 s at order 10) is outside the timings."""
    import torch

    cfg = W.make_config(4)
    c = cfg["cells"]
    lo, hi = c.pos.min(axis=1), c.pos.max(axis=1)
    ctr, R = 0.5 * (lo + hi), 0.5 * float((hi - lo).max()) * 1.0001
    pos, f, w = t(c.pos), t(cfg["f"]), t(c.weight)
    depth = 6
    depths = {4: 6, 6: 6, 8: 5, 10: 5}
    r = {"points": c.n, "depth": depth, "leaves": 8 ** depth, "domain_half_width": R,
         "depth_by_order": {str(k): v for k, v in depths.items()}}
    pick = W.subset(np.random.default_rng(74), c.n, 2000)
    ref = S.sl(pos, f, w, t(c.pos[:, pick])).cpu().numpy()
    out = torch.empty((3, c.n), dtype=torch.float64, device=pos.device)
    for order in (4, 6, 8, 10):
        depth = depths[order]
        t0 = time.perf_counter()
        plan = S.FMMPlan(order)
        torch.cuda.synchronize()
        r[f"order{order}_plan_s"] = time.perf_counter() - t0
        print(f"fmm: order {order} plan ready ({r[f'order{order}_plan_s']:.1f} s)", file=sys.stderr, flush=True)
        for _ in range(warmup):
            S.fmm_sl(plan, pos, f, w, pos, tuple(ctr), R, depth, out=out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            S.fmm_sl(plan, pos, f, w, pos, tuple(ctr), R, depth, out=out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        got = out.cpu().numpy()[:, pick]
        r[f"order{order}_ms"] = ms
        r[f"order{order}_points_per_s"] = c.n / (ms * 1e-3)
        r[f"order{order}_rel_l2_vs_direct"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        S.fmm_sl(plan, pos, f, w, pos, tuple(ctr), R, depth, out=out, precision="mixed")
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            S.fmm_sl(plan, pos, f, w, pos, tuple(ctr), R, depth, out=out, precision="mixed")
        e1.record()
        torch.cuda.synchronize()
        gm = out.cpu().numpy()[:, pick]
        r[f"order{order}_mixed_ms"] = e0.elapsed_time(e1) / steps
        r[f"order{order}_mixed_rel_l2_vs_direct"] = float(np.linalg.norm(gm - ref) / np.linalg.norm(ref))
        r[f"order{order}_mixed_rel_l2_vs_fp64"] = float(np.linalg.norm(gm - got) / np.linalg.norm(got))
        if order == 4:
            # the same evaluation captured once in a HIP graph and replayed (no launch gaps)
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                S.fmm_sl(plan, pos, f, w, pos, tuple(ctr), R, depth, out=out)
            graph.replay()
            torch.cuda.synchronize()
            e0.record()
            for _ in range(steps):
                graph.replay()
            e1.record()
            torch.cuda.synchronize()
            r["order4_graph_ms"] = e0.elapsed_time(e1) / steps
            r["order4_graph_equals_eager"] = bool(np.array_equal(out.cpu().numpy()[:, pick], got))
            del graph
        if order in (6, 10):
            # the same-cell rule of Sec. 2.2: each cell's sum onto itself taken off
            # exactly, against the direct sum with that rule on the same sample
            grp = t(c.group.astype(np.int32))
            ng = int(c.group.max()) + 1
            if order == 6:                                 # the rule's direct reference, once
                ref_ex = S.sl(pos, f, w, t(c.pos[:, pick]), src_group=grp,
                              trg_group=t(c.group[pick].astype(np.int32)), exclude_same_group=True).cpu().numpy()
            S.fmm_sl(plan, pos, f, w, pos, tuple(ctr), R, depth, out=out, src_group=grp, trg_group=grp, n_groups=ng)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(steps):
                S.fmm_sl(plan, pos, f, w, pos, tuple(ctr), R, depth, out=out, src_group=grp, trg_group=grp,
                         n_groups=ng)
            e1.record()
            torch.cuda.synchronize()
            ge = out.cpu().numpy()[:, pick]
            r[f"order{order}_same_cell_ms"] = e0.elapsed_time(e1) / steps
            r[f"order{order}_same_cell_rel_l2_vs_direct"] = float(np.linalg.norm(ge - ref_ex) / np.linalg.norm(ref_ex))
        del plan
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    S.sl(pos, f, w, pos, out=out)
    e1.record()
    torch.cuda.synchronize()
    r["direct_ms"] = e0.elapsed_time(e1)
    r["direct_pairs"] = c.n * c.n
    for order in depths:
        r[f"speedup_order{order}_vs_direct"] = r["direct_ms"] / r[f"order{order}_ms"]
    # the wall's double layer (1,048,576 nodes) at the 522,240 points of 960 cells, order 6
    cfg5 = W.make_config(5)
    wall, cells = cfg5["wall"], cfg5["cells"]
    lo = np.minimum(wall.pos.min(axis=1), cells.pos.min(axis=1))
    hi = np.maximum(wall.pos.max(axis=1), cells.pos.max(axis=1))
    ctr5, R5 = 0.5 * (lo + hi), 0.5 * float((hi - lo).max()) * 1.0001
    args = [t(wall.pos), t(cfg5["phi"]), t(wall.weight), t(wall.normal)]
    cp = t(cells.pos)
    pick5 = W.subset(np.random.default_rng(81), cells.n, 2000)
    ref5 = S.dl(*args, t(cells.pos[:, pick5])).cpu().numpy()
    u5 = torch.empty((3, cells.n), dtype=torch.float64, device=pos.device)
    for order, d5 in ((6, 6), (10, 5)):
        plan = S.FMMPlan(order)
        print(f"fmm: wall double layer, order {order} plan ready", file=sys.stderr, flush=True)
        for _ in range(warmup):
            S.fmm_dl(plan, *args, cp, tuple(ctr5), R5, d5, out=u5)
        e0.record()
        for _ in range(steps):
            S.fmm_dl(plan, *args, cp, tuple(ctr5), R5, d5, out=u5)
        e1.record()
        torch.cuda.synchronize()
        r[f"dl_wall_to_cells_order{order}_depth"] = d5
        r[f"dl_wall_to_cells_order{order}_ms"] = e0.elapsed_time(e1) / steps
        r[f"dl_wall_to_cells_order{order}_rel_l2_vs_direct"] = float(
            np.linalg.norm(u5.cpu().numpy()[:, pick5] - ref5) / np.linalg.norm(ref5))
        e0.record()
        for _ in range(steps):
            S.fmm_dl(plan, *args, cp, tuple(ctr5), R5, d5, out=u5, precision="mixed")
        e1.record()
        torch.cuda.synchronize()
        r[f"dl_wall_to_cells_order{order}_mixed_ms"] = e0.elapsed_time(e1) / steps
        r[f"dl_wall_to_cells_order{order}_mixed_rel_l2_vs_direct"] = float(
            np.linalg.norm(u5.cpu().numpy()[:, pick5] - ref5) / np.linalg.norm(ref5))
        del plan
    e0.record()
    S.dl(*args, cp, out=u5)
    e1.record()
    torch.cuda.synchronize()
    r["dl_wall_to_cells_direct_ms"] = e0.elapsed_time(e1)
    r["dl_wall_to_cells_pairs"] = wall.n * cells.n
    return r


def secondary(S, W, t, timed, log):
    """Timings of the components around the hot path (check points, boundary
    solve, collision candidates, FMM)."""
    out = {}
    r = time_checkpoint(S, W, t, timed, 5, 1, oracle=False)
    out["checkpoint_wall_ring"] = r
    log(f"secondary checkpoint: {r}")
    r = time_bie(S, W, t, 2, 1)
    out["bie_solve_ellipsoid"] = r
    log(f"secondary bie: {r}")
    r = time_collision(S, W, t, 5, 1, oracle=False)
    out["collision_cells_and_wall"] = r
    log(f"secondary collision: {r}")
    r = time_fmm(S, W, t, 2, 1)
    out["fmm_3840_cells"] = r
    log(f"secondary fmm: {r}")
    return out


if __name__ == "__main__":
    main()
