"""Benchmark: cells per second over one flow time step on one MI355X.

Workload (default, --workload plain): the synthetic 19-species /
50-reversible-reaction field of 262 144 cells (70 % at T ~ U[300, 900] K,
30 % at T ~ U[1400, 2500] K, Dirichlet mass fractions, 1 atm), integrated
over dt_flow = 1e-4 s in FP64.  A step is one stev_integrate call over the
whole field (inputs already resident in HBM); before each step the initial
state is restored on the device.  Prints one JSON line.

Other workloads (one JSON line each, same keys):
  --workload batched  64 batches, log-uniform sizes in [256, 131072],
                      alternating 6- and 19-species mechanisms, FP32, one
                      stev_integrate_batched call per step (graph replay,
                      autotuned launch shape), against 64 plain calls
  --workload mlp      19 species, 1 048 576 cells, FP32 with the thermo
                      network against FP32 polynomials
  --workload c3m      the multiphase C3M gasification chemistry (Sec 7.2):
                      262 144 random gas-solid cells of 26 values,
                      dt_flow = 1e-3 s
  --workload serve    Poisson arrivals of requests of log-uniform size in
                      [1024, 524288] cells over 6-, 19- and 53-species
                      mechanisms, FP32 + thermo network, host-resident
                      requests admitted by an HBM budget that binds; p50/p99
                      latency against plain per-request launches

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision f64|f32]
                  [--workload plain|batched|mlp|serve|c3m]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cells/sec over one flow Δt, plain vs batched+MLP STEV; p50/p99 solve latency"
PEAK = {"f64": 78.6, "f32": 157.3}   # TFLOP/s, MI355X vector FP64 / FP32
KERNEL_SOURCES = ["paper_1905_09395_amd/csrc/stev_kernel.hip",
                  "paper_1905_09395_amd/csrc/stev_persistent.h",
                  "paper_1905_09395_amd/csrc/stev_math.h",
                  "paper_1905_09395_amd/csrc/stev_internal.h",
                  "paper_1905_09395_amd/csrc/stev_thermo.h",
                  "paper_1905_09395_amd/csrc/stev_variants.h"]


def kernel_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        with open(os.path.join(ROOT, s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(precision, cells):
    """HBM bytes per launch from the committed FETCH_SIZE/WRITE_SIZE summary,
    or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"stev_traffic_{precision}_mech19_{cells}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_sources_sha256") != kernel_sources_sha():
        return None
    return rec["traffic_bytes_per_launch"]


def traffic_probe(precision):
    """One plain copy of known size (counter calibration), then one step."""
    import torch
    n = PROBE_COPY_BYTES // 4
    x = torch.ones(n, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(f"probe: copy of {n * 4} bytes read and {n * 4} bytes written", flush=True)


def cpu_baseline(mech, T, P, Y, dt, budget_s=12.0):
    """Time the FP64 CPU oracle (as it stands) on a bounded seeded sample."""
    import numpy as np

    import oracle
    from paper_1905_09395_amd import synth
    om = oracle.OracleMech(mech)
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    n = 64
    total_cells, total_s = 0, 0.0
    seed = 900
    while total_s < budget_s and n <= 65536:
        idx = synth.subsample(len(T), n, seed=seed)
        seed += 1
        t0 = time.perf_counter()
        oracle.integrate(om, T[idx], P[idx], Y[idx], dt, nthreads=cores)
        el = time.perf_counter() - t0
        total_cells += n
        total_s += el
        if el < budget_s / 4:
            n *= 2
    # the same recipe on one thread, over a smaller sample
    n1, cells1, s1, seed1 = 16, 0, 0.0, 950
    while s1 < budget_s / 4 and n1 <= 4096:
        idx = synth.subsample(len(T), n1, seed=seed1)
        seed1 += 1
        t0 = time.perf_counter()
        oracle.integrate(om, T[idx], P[idx], Y[idx], dt, nthreads=1)
        el = time.perf_counter() - t0
        cells1 += n1
        s1 += el
        if el < budget_s / 16:
            n1 *= 2
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": total_cells / total_s, "unit": "cells/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{total_cells} cells drawn (seeded, without replacement) from the same "
                      f"{len(T)}-cell field in batches of doubling size, {total_s:.1f} s of "
                      f"FP64 oracle time with OpenMP over {cores} host threads",
            "one_thread_value": cells1 / s1,
            "one_thread_sample": f"{cells1} cells drawn the same way, {s1:.1f} s on one thread",
            "cpu_model": model}


PROBE_COPY_BYTES = 64 * 1024 * 1024 * 4


def traffic_summary(fetch_csv, write_csv, precision, cells):
    """Turn two rocprofv3 --pmc runs of `bench.py --probe` (FETCH_SIZE, then
    WRITE_SIZE; KiB per dispatch) into HBM bytes per integration launch,
    each counter scaled by what it reads for the probe's plain copy of known
    size.  Writes profiles/stev_traffic_<prec>_mech19_<cells>.json and .md."""
    import csv

    def read(path, counter):
        # the integration launch is the last stev_persistent dispatch of the
        # step (a probe launch of the dispatch-order refinement precedes it)
        copy, stev = [], {}
        with open(path) as f:
            for row in csv.DictReader(f):
                if row["Counter_Name"] != counter:
                    continue
                v = float(row["Counter_Value"])
                if "copyBuffer" in row["Kernel_Name"]:
                    copy.append(v)
                elif "stev_persistent" in row["Kernel_Name"]:
                    d = int(row["Dispatch_Id"])
                    stev[d] = stev.get(d, 0.0) + v
        assert copy and 1 <= len(stev) <= 2, f"{path}: expected copies and the step's launches"
        return max(copy), stev[max(stev)]

    fc, fs = read(fetch_csv, "FETCH_SIZE")
    wc, ws = read(write_csv, "WRITE_SIZE")
    kib = PROBE_COPY_BYTES / 1024.0
    f_fac, w_fac = kib / fc, kib / wc
    fetch_b = fs * f_fac * 1024.0
    write_b = ws * w_fac * 1024.0
    rsz = 8 if precision == "f64" else 4
    algo = cells * (2 * 19 + 3) * rsz
    rec = {"kernel": "stev_persistent", "precision": precision, "cells": cells,
           "fetch_kib_raw": fs, "write_kib_raw": ws,
           "copy_fetch_kib_raw": fc, "copy_write_kib_raw": wc,
           "fetch_scale": f_fac, "write_scale": w_fac,
           "fetch_bytes": fetch_b, "write_bytes": write_b,
           "traffic_bytes_per_launch": fetch_b + write_b,
           "algorithmic_bytes_per_launch": algo,
           "kernel_sources_sha256": kernel_sources_sha(),
           "commands": [
               f"rocprofv3 --pmc FETCH_SIZE -d gpurun_out/pmc_fetch_{precision} -o t "
               f"--output-format csv -- python bench.py --probe --precision {precision}",
               f"rocprofv3 --pmc WRITE_SIZE -d gpurun_out/pmc_write_{precision} -o t "
               f"--output-format csv -- python bench.py --probe --precision {precision}",
               f"python bench.py --traffic-summary gpurun_out/pmc_fetch_{precision}/t_counter_collection.csv "
               f"gpurun_out/pmc_write_{precision}/t_counter_collection.csv --precision {precision}"]}
    base = os.path.join(ROOT, "profiles", f"stev_traffic_{precision}_mech19_{cells}")
    with open(base + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    with open(base + ".md", "w") as f:
        f.write(f"# HBM traffic of one stev_persistent launch ({precision}, 19 species, "
                f"{cells} cells)\n\n")
        f.write("Commands (committed files only):\n\n")
        for c in rec["commands"]:
            f.write(f"    {c}\n")
        f.write(f"\n| quantity | value |\n|---|---|\n")
        f.write(f"| FETCH_SIZE, launch (KiB, raw) | {fs:.0f} |\n")
        f.write(f"| WRITE_SIZE, launch (KiB, raw) | {ws:.0f} |\n")
        f.write(f"| copy of {PROBE_COPY_BYTES} B: FETCH_SIZE / WRITE_SIZE (KiB, raw) | "
                f"{fc:.0f} / {wc:.0f} |\n")
        f.write(f"| scale FETCH / WRITE | {f_fac:.3f} / {w_fac:.3f} |\n")
        f.write(f"| read + written per launch (MB) | {fetch_b / 1e6:.1f} + {write_b / 1e6:.1f} |\n")
        f.write(f"| algorithmic state bytes (MB) | {algo / 1e6:.1f} |\n")
    print(json.dumps(rec))


def pmc_summary(csv_paths, precision, cells):
    """Summarise rocprofv3 --pmc runs of `bench.py --probe` (counters of the
    one integration launch) into profiles/stev_pmc_<prec>_mech19_<cells>.md."""
    import csv
    vals = {}
    for path in csv_paths:
        per = {}   # dispatch -> counters; the integration launch is the last
        with open(path) as f:
            for row in csv.DictReader(f):
                if "stev_persistent" in row["Kernel_Name"]:
                    c = per.setdefault(int(row["Dispatch_Id"]), {})
                    c[row["Counter_Name"]] = c.get(row["Counter_Name"], 0.0) + float(row["Counter_Value"])
        if per:
            vals.update(per[max(per)])
    base = os.path.join(ROOT, "profiles", f"stev_pmc_{precision}_mech19_{cells}")
    with open(base + ".md", "w") as f:
        f.write(f"# Counters of one stev_persistent launch ({precision}, 19 species, {cells} cells)\n\n")
        f.write("Each counter set from its own run of:\n\n")
        sets = {"f64": [("valu_f64", "SQ_INSTS_VALU_FLOPS_FP64 SQ_INSTS_VALU_FLOPS_FP64_TRANS "
                                     "SQ_INSTS_VALU SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_ADD_F64 "
                                     "SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_TRANS_F64 SQ_INSTS_LDS"),
                        ("cyc_f64", "SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY "
                                    "SQ_ACTIVE_INST_ANY SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS "
                                    "SQ_INSTS_SALU")],
                "f32": [("valu_f32", "SQ_INSTS_VALU_FLOPS_FP32 SQ_INSTS_VALU_FLOPS_FP32_TRANS "
                                     "SQ_INSTS_VALU SQ_INSTS_VALU_FMA_F32 SQ_INSTS_VALU_ADD_F32 "
                                     "SQ_INSTS_VALU_MUL_F32 SQ_INSTS_VALU_TRANS_F32 SQ_INSTS_LDS"),
                        ("cyc_f32", "SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY "
                                    "SQ_ACTIVE_INST_ANY SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS "
                                    "SQ_INSTS_SALU")]}
        for name, ctrs in sets[precision]:
            f.write(f"    rocprofv3 --pmc {ctrs} -d gpurun_out/pmc_{name} -o t --output-format csv "
                    f"-- python bench.py --probe --precision {precision}\n")
        f.write("    python bench.py --pmc-summary " +
                " ".join(f"gpurun_out/pmc_{name}/t_counter_collection.csv" for name, _ in sets[precision]) +
                f" --precision {precision}\n\n")
        f.write("| counter | value |\n|---|---|\n")
        for k in sorted(vals):
            f.write(f"| {k} | {vals[k]:.6g} |\n")
        fl = "FP64" if precision == "f64" else "FP32"
        key = f"SQ_INSTS_VALU_FLOPS_{fl}"
        if key in vals:
            f.write(f"\nCounted VALU FLOP per launch = 64 lanes x {key} "
                    f"(ADD + MUL + 2 FMA + TRANS per wave instruction) = "
                    f"{64 * vals[key]:.4g}; this counts every lane of every issued "
                    f"instruction, idle lanes and software exp/log/divide included.\n")
    rec = {"kernel": "stev_persistent", "precision": precision, "cells": cells,
           "counters": vals, "kernel_sources_sha256": kernel_sources_sha()}
    with open(base + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(vals))


def counted_flops(precision, cells):
    """Issued VALU lane-FLOP per launch from rocprofv3 counters (64 lanes x
    (ADD + MUL + 2 FMA + TRANS) instructions, every lane counted whether
    active or not), from the committed counter record, or None when the
    kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"stev_pmc_{precision}_mech19_{cells}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_sources_sha256") != kernel_sources_sha():
        return None
    key = "SQ_INSTS_VALU_FLOPS_" + ("FP64" if precision == "f64" else "FP32")
    v = rec["counters"].get(key)
    return None if v is None else 64.0 * v


def direct_dft_flops(mech):
    """FLOP per cell-iteration with the 13-point DFT counted as direct sums:
    10 + 51 n_s + sum over reactions of (15 + 4 p) if reversible, (7 + 2 p)
    otherwise (p participants), + 185 per reversible reaction for the ring's
    |DFT| at bins 0 and 4..6 (add/mul = 1, FMA = 2).  This is the count the
    roofline fraction uses; the library's own stev_model_flops counts the
    pair-symmetric DFT the kernels evaluate (70 per reversible reaction)."""
    import numpy as np
    ptr = np.asarray(mech["rxn_ptr"])
    rev = np.asarray(mech["reversible"]).astype(bool)
    p = np.diff(ptr)
    return float(10 + 51 * int(mech["n_s"]) + np.sum(np.where(rev, 15 + 4 * p, 7 + 2 * p))
                 + 185 * int(rev.sum()))


def base_record(args, value, el, dtype, workload, **config):
    return {"metric": METRIC, "value": value, "unit": "cells/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": el * 1e3 / args.steps,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": dict(workload=workload, **config)}


def run_batched(args):
    """64 uneven batches per step in one stev_integrate_batched call."""
    import numpy as np
    import torch

    from paper_1905_09395_amd import stev, synth
    dev = torch.device("cuda:0")
    dt = 1e-4
    batches = synth.make_batches(64, 256, 131072, seed=103)
    ctx = stev.Context(0)
    ctx.set_stream(torch.cuda.current_stream(dev))
    mechs = {6: ctx.mechanism(synth.make_mech6()), 19: ctx.mechanism(synth.make_mech19())}
    prec = stev.F32
    f32 = torch.float32
    B = [dict(key=k, T0=torch.tensor(T, dtype=f32, device=dev),
              P=torch.tensor(P, dtype=f32, device=dev),
              Y0=torch.tensor(Y, dtype=f32, device=dev).contiguous(),
              it=torch.zeros(len(T), dtype=torch.int32, device=dev)) for k, T, P, Y in batches]
    for b in B:
        b["T"], b["Y"] = b["T0"].clone(), b["Y0"].clone()
    n_cells = sum(len(b[1]) for b in batches)
    # autotuned launch shape per mechanism (on that mechanism's cells), outside
    # the timed region
    tuned = {}
    for k, gm in mechs.items():
        sel = [b for b in B if b["key"] == k]
        Tc = torch.cat([b["T0"] for b in sel])
        Pc = torch.cat([b["P"] for b in sel])
        Yc = torch.cat([b["Y0"] for b in sel])
        tuned[k] = ctx.autotune(gm, Tc, Pc, Yc, dt, stev.default_params(precision=prec))
    # the call leaves the launch shape on auto: each mechanism's launch takes
    # the shape tuned (and cached in the context) for it
    prm = stev.default_params(precision=prec)

    def restore():
        for b in B:
            b["T"].copy_(b["T0"])
            b["Y"].copy_(b["Y0"])

    def step_batched():
        restore()
        return ctx.integrate_batched([mechs[b["key"]] for b in B], [b["T"] for b in B],
                                     [b["P"] for b in B], [b["Y"] for b in B], dt, params=prm,
                                     iters=[b["it"] for b in B])[1]

    def step_plain():
        restore()
        ms = 0.0
        for b in B:
            ms += ctx.integrate(mechs[b["key"]], b["T"], b["P"], b["Y"], dt,
                                params=stev.default_params(precision=prec))[1]["kernel_ms"]
        return ms

    for _ in range(args.warmup):
        step_batched()
        step_plain()
    torch.cuda.synchronize()
    # per-mechanism iteration totals (deterministic) for the model FLOPs
    step_batched()
    torch.cuda.synchronize()
    work = work_pair = 0.0
    for k, gm in mechs.items():
        its = sum(int(b["it"].sum().item()) for b in B if b["key"] == k)
        work += its * direct_dft_flops(gm.mech)
        work_pair += its * gm.model_flops(stev.THERMO_POLY)[0]
    t0 = time.perf_counter()
    kms = []
    for _ in range(args.steps):
        kms.append(step_batched()["kernel_ms"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    t1 = time.perf_counter()
    pms = []
    for _ in range(args.steps):
        pms.append(step_plain())
    torch.cuda.synchronize()
    el_plain = time.perf_counter() - t1
    k_ms = float(np.mean(kms))
    achieved = work / (k_ms * 1e-3) / 1e12

    # accuracy: every cell against the same batches in FP64 (polynomials)
    def rel_T():
        return np.concatenate([b["T"].cpu().double().numpy() for b in B])
    f64 = torch.float64
    R = [dict(T=torch.tensor(T, dtype=f64, device=dev), P=torch.tensor(P, dtype=f64, device=dev),
              Y=torch.tensor(Y, dtype=f64, device=dev).contiguous()) for k, T, P, Y in batches]
    ctx.integrate_batched([mechs[b["key"]] for b in B], [r["T"] for r in R], [r["P"] for r in R],
                          [r["Y"] for r in R], dt, params=stev.default_params(precision=stev.F64))
    refT = np.concatenate([r["T"].cpu().numpy() for r in R])
    del R
    step_batched()
    torch.cuda.synchronize()
    err_poly = np.abs(rel_T() - refT) / refT

    # batched with the thermo network (trained per mechanism, launch shape
    # tuned per mechanism for that thermo mode)
    for k, gm in mechs.items():
        ctx.train_thermo_mlp(gm, epochs=300, n_samples=1 << 20, batch=8192, lr=3e-3, seed=104)
        sel = [b for b in B if b["key"] == k]
        ctx.autotune(gm, torch.cat([b["T0"] for b in sel]), torch.cat([b["P"] for b in sel]),
                     torch.cat([b["Y0"] for b in sel]), dt,
                     stev.default_params(precision=prec, thermo=stev.THERMO_MLP))
    prm_mlp = stev.default_params(precision=prec, thermo=stev.THERMO_MLP)

    def step_batched_mlp():
        restore()
        return ctx.integrate_batched([mechs[b["key"]] for b in B], [b["T"] for b in B],
                                     [b["P"] for b in B], [b["Y"] for b in B], dt,
                                     params=prm_mlp, iters=[b["it"] for b in B])[1]

    for _ in range(args.warmup):
        step_batched_mlp()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        step_batched_mlp()
    torch.cuda.synchronize()
    el_mlp = time.perf_counter() - t2
    err_mlp = np.abs(rel_T() - refT) / refT

    out = base_record(args, n_cells * args.steps / el, el, "f32",
                      "batched STEV: 64 batches of log-uniform size in [256, 131072], "
                      "alternating 6-species/4-reaction and 19-species/50-reaction "
                      "mechanisms, one persistent launch per mechanism, graph replay, "
                      "autotuned launch shape, FP32, dt_flow=1e-4 s; beside it the same "
                      "batches with the tanh thermo network and as 64 plain calls",
                      cells=n_cells, batches=64,
                      tuned={str(k): dict(lanes_per_cell=v.lanes_per_cell,
                                          waves_per_wg=v.waves_per_wg,
                                          compact_every=v.compact_every)
                             for k, v in tuned.items()},
                      plain_per_batch_cells_per_s=n_cells * args.steps / el_plain,
                      plain_per_batch_kernel_ms=float(np.mean(pms)),
                      speedup_vs_plain_per_batch=el_plain / el,
                      batched_network_cells_per_s=n_cells * args.steps / el_mlp,
                      batched_network_speedup_vs_plain_per_batch=el_plain / el_mlp,
                      rel_T_vs_fp64=dict(
                          batched_poly=dict(median=float(np.median(err_poly)),
                                            p99=float(np.quantile(err_poly, .99))),
                          batched_network=dict(median=float(np.median(err_mlp)),
                                               p99=float(np.quantile(err_mlp, .99)))))
    out["roofline"] = {"bound": "alu", "achieved": achieved, "peak": PEAK["f32"],
                       "unit": "TFLOP/s", "frac": achieved / PEAK["f32"], "traffic": None,
                       "kernel_ms": k_ms, "flop_count": "direct 13-point DFT",
                       "frac_pair_symmetric_dft": work_pair / (k_ms * 1e-3) / 1e12 / PEAK["f32"]}
    ctx.close()
    return out


def run_mlp(args):
    """1 048 576 cells of the 19-species field, FP32, thermo network vs polynomials."""
    import numpy as np
    import torch

    from paper_1905_09395_amd import stev, synth
    dev = torch.device("cuda:0")
    dt = 1e-4
    n = 1 << 20
    mech = synth.make_mech19()
    T, P, Y = synth.make_cells_mech19(n, seed=104)
    ctx = stev.Context(0)
    ctx.set_stream(torch.cuda.current_stream(dev))
    gm = ctx.mechanism(mech)
    rep = ctx.train_thermo_mlp(gm, epochs=300, n_samples=1 << 20, batch=8192, lr=3e-3, seed=104)
    # the paper's own network: one sigmoid layer as wide as the outputs,
    # fitted by Levenberg-Marquardt
    lrep, lprm = ctx.train_thermo_lma(gm, iters=150, n_samples=1 << 16, seed=104)
    ctx.set_thermo_ann(gm, lrep["hidden"], 300.0, 3000.0, lprm)
    f32 = torch.float32
    T0 = torch.tensor(T, dtype=f32, device=dev)
    P0 = torch.tensor(P, dtype=f32, device=dev)
    Y0 = torch.tensor(Y, dtype=f32, device=dev).contiguous()
    Tw, Yw = T0.clone(), Y0.clone()
    # accuracy reference: the FP64 polynomial path on the same field (its
    # parity with the FP64 oracle is what the tests establish)
    f64 = torch.float64
    Tr = torch.tensor(T, dtype=f64, device=dev)
    Yr = torch.tensor(Y, dtype=f64, device=dev).contiguous()
    ctx.integrate(gm, Tr, torch.tensor(P, dtype=f64, device=dev), Yr, dt,
                  params=stev.default_params(precision=stev.F64))
    refT = Tr.cpu().numpy()
    refY = Yr.cpu().numpy()
    del Tr, Yr
    res = {}
    for name, th in (("network", stev.THERMO_MLP), ("sigmoid", stev.THERMO_ANN),
                     ("poly", stev.THERMO_POLY)):
        # the launch shape the autotuner picks for this thermo mode and field
        # (outside the timed region), beside the default shape
        prm = ctx.autotune(gm, T0, P0, Y0, dt, stev.default_params(precision=stev.F32, thermo=th))
        shape = dict(lanes_per_cell=prm.lanes_per_cell, waves_per_wg=prm.waves_per_wg,
                     compact_every=prm.compact_every)
        base = stev.default_params(precision=stev.F32, thermo=th)
        base_ms = []
        for _ in range(max(1, args.steps // 2)):
            Tw.copy_(T0); Yw.copy_(Y0)
            base_ms.append(ctx.integrate(gm, Tw, P0, Yw, dt, params=base)[1]["kernel_ms"])
        for _ in range(args.warmup):
            Tw.copy_(T0); Yw.copy_(Y0)
            ctx.integrate(gm, Tw, P0, Yw, dt, params=prm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kms, lms, its = [], [], []
        for _ in range(args.steps):
            Tw.copy_(T0); Yw.copy_(Y0)
            st = ctx.integrate(gm, Tw, P0, Yw, dt, params=prm)[1]
            kms.append(st["kernel_ms"]); lms.append(st["launch_ms"]); its.append(st["total_iters"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        # accuracy of every cell against the FP64 polynomial result
        gT = Tw.cpu().double().numpy()
        gY = Yw.cpu().double().numpy()
        m = refY > 1e-6
        relT = np.abs(gT - refT) / refT
        relY = np.where(m, np.abs(gY - refY) / np.where(m, refY, 1), 0).max(axis=1)
        res[name] = dict(el=el, kms=float(np.mean(kms)), launch_ms=float(np.mean(lms)),
                         its=float(np.mean(its)),
                         tuned_shape=shape, default_shape_kernel_ms=float(np.mean(base_ms)),
                         median_rel_T=float(np.median(relT)), p99_rel_T=float(np.quantile(relT, .99)),
                         median_rel_Y=float(np.median(relY)), p99_rel_Y=float(np.quantile(relY, .99)))
    flops = direct_dft_flops(mech)
    r = res["network"]
    # the integration launch alone, as for the plain workload (kms adds the
    # probe and ordering kernels of the same call)
    achieved = r["its"] * flops / (r["launch_ms"] * 1e-3) / 1e12
    out = base_record(args, n * args.steps / r["el"], r["el"], "f32",
                      "learned thermo: 19-species/50-reaction mechanism, 1048576 cells, FP32, "
                      "cp and h from a 1-32-32-38 tanh network (bf16 MFMA, fp32 accumulation, "
                      "polynomial fallback outside 300-3000 K), dt_flow=1e-4 s, autotuned launch "
                      "shape for each thermo mode; beside it the paper's 1-38-38 sigmoid "
                      "network (FP32 vector units) and the polynomials",
                      cells=n, network_train=dict(test_loss=rep["test_loss"],
                                                  max_rel_err_cp=rep["max_rel_err_cp"],
                                                  max_rel_err_h=rep["max_rel_err_h"],
                                                  train_ms=rep["train_ms"]),
                      network=dict((k, v) for k, v in r.items() if k != "el"),
                      sigmoid_network=dict((k, v) for k, v in res["sigmoid"].items() if k != "el"),
                      sigmoid_train=dict(hidden=lrep["hidden"], test_loss=lrep["test_loss"],
                                         max_rel_err_cp=lrep["max_rel_cp"],
                                         train_ms=lrep["train_ms"]),
                      polynomials=dict((k, v) for k, v in res["poly"].items() if k != "el"),
                      poly_cells_per_s=n * args.steps / res["poly"]["el"],
                      sigmoid_cells_per_s=n * args.steps / res["sigmoid"]["el"],
                      network_over_poly_time=r["el"] / res["poly"]["el"],
                      sigmoid_over_poly_time=res["sigmoid"]["el"] / res["poly"]["el"],
                      accuracy_sample="every cell vs the FP64 polynomial path on the GPU; "
                                      "relative errors, Y over Y_k > 1e-6")
    out["roofline"] = {"bound": "alu", "achieved": achieved, "peak": PEAK["f32"],
                       "unit": "TFLOP/s", "frac": achieved / PEAK["f32"], "traffic": None,
                       "kernel_ms": r["launch_ms"], "call_kernel_ms": r["kms"],
                       "flop_count": "direct 13-point DFT, network evaluation not counted"}
    ctx.close()
    return out


def run_c3m(args):
    """The multiphase C3M gasification field: 262 144 random gas-solid cells
    (26 values each), integrated over dt_flow = 1e-3 s."""
    import numpy as np
    import torch

    from paper_1905_09395_amd import stev, synth
    dev = torch.device("cuda:0")
    dt = 1e-3
    n = args.cells
    desc = synth.make_c3m()
    st = synth.make_c3m_cells(n, seed=108)
    ctx = stev.Context(0)
    ctx.set_stream(torch.cuda.current_stream(dev))
    g = ctx.c3m(desc)
    prec = stev.F64 if args.precision == "f64" else stev.F32
    dtype = torch.float64 if prec == stev.F64 else torch.float32
    S0 = torch.tensor(st, dtype=dtype, device=dev)
    Sw = S0.clone()
    prm = stev.default_params(precision=prec)

    def step():
        Sw.copy_(S0)
        return ctx.c3m_integrate(g, Sw, dt, params=prm)[1]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    kms, its = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = step()
        kms.append(r["launch_ms"])
        its.append(r["total_iters"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    flops, transc = g.model_flops()
    k_ms = float(np.mean(kms))
    achieved = float(np.mean(its)) * flops / (k_ms * 1e-3) / 1e12
    rsz = 8 if prec == stev.F64 else 4
    out = base_record(args, n * args.steps / el, el, args.precision,
                      f"multiphase C3M gasification (Sec 7.2, Eqs 31-56, Table 2): {n} random "
                      f"gas-solid cells of 26 values (T_g 900-1400 K, P 1-15 atm, eps_s "
                      f"0.02-0.3, d_p 50-500 um, Dirichlet gas and solid fractions), "
                      f"dt_flow=1e-3 s, {args.precision}",
                      cells=n, dt_flow=dt, lanes_per_cell=1, waves_per_wg=r["waves_per_wg"],
                      grid_wgs=r["grid_wgs"],
                      cell_iterations_per_step=int(np.mean(its)),
                      max_cell_iterations=r["max_cell_iters"],
                      load_curve=stev.load_curve(r["load_hist"]))
    out["roofline"] = {"bound": "alu", "achieved": achieved, "peak": PEAK[args.precision],
                       "unit": "TFLOP/s", "frac": achieved / PEAK[args.precision],
                       "traffic": None, "kernel_ms": k_ms,
                       "model_flop_per_cell_iter": flops,
                       "transcendentals_per_cell_iter": transc,
                       "state_bytes_per_launch": 2 * 26 * rsz * n}
    if not args.no_cpu:   # the cpu_baseline leg: the oracle timed as it stands
        import oracle
        cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
        oc = oracle.C3M(desc)
        m, tot_c, tot_s, seed = 256, 0, 0.0, 900
        while tot_s < 12.0 and m <= 65536:
            idx = synth.subsample(n, m, seed=seed)
            seed += 1
            t1 = time.perf_counter()
            oracle.c3m_integrate(oc, st[idx], dt, nthreads=cores)
            e = time.perf_counter() - t1
            tot_c += m
            tot_s += e
            if e < 3.0:
                m *= 2
        out["cpu_baseline"] = {"value": tot_c / tot_s, "unit": "cells/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"{tot_c} cells drawn (seeded) from the same field in "
                                         f"batches of doubling size, {tot_s:.1f} s of FP64 "
                                         f"oracle time over {cores} host threads"}
    g.close()
    ctx.close()
    return out


def run_serve(args):
    """Poisson-arrival serving against plain per-request launches."""
    import threading

    import numpy as np
    import torch

    from paper_1905_09395_amd import stev, synth
    dt = 1e-4
    rng = np.random.default_rng(105)
    n_req = 32
    sizes = np.round(np.exp(rng.uniform(np.log(1024), np.log(524288), n_req))).astype(int)
    keys = rng.choice([6, 19, 53], n_req)
    mean_cells = 83879.0
    src = {6: synth.make_mech6(), 19: synth.make_mech19(), 53: synth.make_mech53()}
    n_s = {6: 6, 19: 19, 53: 53}
    # host-resident (pinned) request state; the serving context stages it
    # through a device budget of the largest request's staging plus 48 MiB
    # (mechanisms, networks, launch tables, dispatch orders and the smaller
    # requests), so that admission binds whenever a large request is in
    # flight and another arrives.  The plain baseline runs in a context of its
    # own (default budget), and the networks are trained there and imported
    # into the serving context.
    stage = [int(n) * (2 + n_s[int(k)] + 1) * 4 for k, n in zip(keys, sizes)]
    budget = max(stage) + (48 << 20)
    plain = stev.Context(0)
    ctx = stev.Context(0, hbm_budget=budget)
    mechs, pmechs = {}, {}
    for k, m in src.items():
        pm = plain.mechanism(m)
        plain.train_thermo_mlp(pm, epochs=100, n_samples=1 << 20, batch=4096, lr=3e-3, seed=104)
        pmechs[k] = pm
        mechs[k] = ctx.mechanism(m)
        ctx.set_thermo_mlp(mechs[k], 32, 300.0, 3000.0, plain.get_thermo_mlp(pm))
    prm = stev.default_params(precision=stev.F32, thermo=stev.THERMO_MLP)

    def make(k, n, seed):
        T, P, Y = synth.make_cells_mech6(n, seed) if k == 6 else synth.make_cells_split(n, k, seed)
        pin = lambda a: torch.tensor(a, dtype=torch.float32).pin_memory()
        return dict(k=int(k), T0=pin(T), P=pin(P), Y0=pin(Y), T=pin(T), Y=pin(Y))

    reqs = [make(k, n, 50000 + i) for i, (k, n) in enumerate(zip(keys, sizes))]
    total = int(sizes.sum())

    def reset():
        for r in reqs:
            r["T"].copy_(r["T0"]); r["Y"].copy_(r["Y0"])

    # capacity: plain per-request launches back to back
    reset()
    t0 = time.perf_counter()
    for r in reqs:
        plain.integrate(pmechs[r["k"]], r["T"], r["P"], r["Y"], dt, params=prm)
    cap = total / (time.perf_counter() - t0)
    print(f"serve: {n_req} requests, {total} cells; plain capacity {cap:.0f} cells/s",
          file=sys.stderr, flush=True)

    def arrivals(load):
        lam = load * cap / mean_cells
        return np.cumsum(np.random.default_rng(7).exponential(1.0 / lam, n_req))

    def serve_run(at, ctx=ctx, mechs=mechs):
        import queue
        reset()
        lat = [None] * n_req
        waits = [0] * n_req
        submitted = queue.Queue()
        start = time.perf_counter()

        def submitter():
            for i, r in enumerate(reqs):
                d = at[i] - (time.perf_counter() - start)
                if d > 0:
                    time.sleep(d)
                submitted.put((ctx.submit(mechs[r["k"]], r["T"], r["P"], r["Y"], dt,
                                          params=prm), i))

        th = threading.Thread(target=submitter)
        th.start()
        pending = {}
        n_done = 0
        while n_done < n_req:
            while not submitted.empty():
                tk, i = submitted.get()
                pending[tk] = i
            for tk in list(pending):
                rc, st = ctx.poll(tk)
                if rc != stev.STEV_EAGAIN:
                    i = pending.pop(tk)
                    lat[i] = (time.perf_counter() - start) - at[i]
                    waits[i] = st["budget_waits"]
                    n_done += 1
            time.sleep(1e-4)
        th.join()
        makespan = time.perf_counter() - start
        return np.array(lat), makespan, int(np.sum(np.array(waits) > 0))

    def plain_run(at):
        reset()
        lat = np.zeros(n_req)
        start = time.perf_counter()
        for i, r in enumerate(reqs):
            d = at[i] - (time.perf_counter() - start)
            if d > 0:
                time.sleep(d)
            plain.integrate(pmechs[r["k"]], r["T"], r["P"], r["Y"], dt, params=prm)
            lat[i] = (time.perf_counter() - start) - at[i]
        return lat, time.perf_counter() - start

    rows = {}
    for load in (0.5, 0.8, 0.95, "saturated"):
        at = np.zeros(n_req) if load == "saturated" else arrivals(load)
        for _ in range(args.warmup):
            serve_run(at)
        # served and plain runs alternate, the same number of each, so that
        # both quantiles come from equally many samples
        ls, ms, bw, lps, mps = [], [], [], [], []
        for _ in range(args.steps):
            l, m, w = serve_run(at)
            ls.append(l); ms.append(m); bw.append(w)
            l, m = plain_run(at)
            lps.append(l); mps.append(m)
        print(f"serve: load {load} done", file=sys.stderr, flush=True)
        L, LP = np.concatenate(ls), np.concatenate(lps)
        big = int(np.argmax(sizes * np.array([n_s[int(k)] ** 2 for k in keys])))
        rows[str(load)] = dict(
            serve_p50_ms=1e3 * float(np.quantile(L, .5)), serve_p99_ms=1e3 * float(np.quantile(L, .99)),
            serve_max_ms=1e3 * float(L.max()),
            serve_cells_per_s=total / float(np.mean(ms)),
            requests_that_waited_for_budget=int(np.max(bw)),
            plain_p50_ms=1e3 * float(np.quantile(LP, .5)), plain_p99_ms=1e3 * float(np.quantile(LP, .99)),
            plain_max_ms=1e3 * float(LP.max()),
            plain_cells_per_s=total / float(np.mean(mps)),
            # the costliest request (most cells x species^2): its latency in
            # each mode, mean over the runs
            costliest_request_serve_ms=1e3 * float(np.mean([l[big] for l in ls])),
            costliest_request_plain_ms=1e3 * float(np.mean([l[big] for l in lps])))
    # the same load 0.95 arrivals under a budget that admits the largest
    # request with 4 MiB to spare: admission then binds whenever a large
    # request is in flight (requests queue for memory, at a latency cost)
    tight = max(stage) + (4 << 20)
    ctx_t = stev.Context(0, hbm_budget=tight)
    mechs_t = {}
    for k, m in src.items():
        mechs_t[k] = ctx_t.mechanism(m)
        ctx_t.set_thermo_mlp(mechs_t[k], 32, 300.0, 3000.0, plain.get_thermo_mlp(pmechs[k]))
    at = arrivals(0.95)
    for _ in range(args.warmup):
        serve_run(at, ctx_t, mechs_t)
    ls, ms_t, bw = [], [], []
    for _ in range(args.steps):
        l, m, w = serve_run(at, ctx_t, mechs_t)
        ls.append(l); ms_t.append(m); bw.append(w)
    L = np.concatenate(ls)
    rows["0.95_tight_budget"] = dict(
        hbm_budget_bytes=tight,
        serve_p50_ms=1e3 * float(np.quantile(L, .5)), serve_p99_ms=1e3 * float(np.quantile(L, .99)),
        serve_max_ms=1e3 * float(L.max()), serve_cells_per_s=total / float(np.mean(ms_t)),
        requests_that_waited_for_budget=int(np.max(bw)))
    print("serve: tight budget done", file=sys.stderr, flush=True)
    ctx_t.close()
    top = rows["0.95"]
    out = base_record(args, top["serve_cells_per_s"], float(np.sum(ms)), "f32",
                      "serving: Poisson arrivals, 32 requests of log-uniform size in "
                      "[1024, 524288] cells over 6-, 19- and 53-species mechanisms, FP32 + "
                      "thermo network, host-resident pinned requests admitted by an HBM budget "
                      "of the largest request's staging + 48 MiB; value at load 0.95 "
                      "('saturated': every request at t=0; '0.95_tight_budget': the load 0.95 "
                      "arrivals with a budget of the largest staging + 4 MiB); quantiles over "
                      "the same number of served and plain runs",
                      requests=n_req, cells=total, hbm_budget_bytes=budget,
                      plain_capacity_cells_per_s=cap, loads=rows)
    ctx.close()
    plain.close()
    return out


def run_solo(args):
    """Latency of one iteration of the field's slowest cell integrated alone
    (one wavefront on an otherwise idle GPU): the quantity that bounds the
    field's launch, whose length is that cell's iteration count times it."""
    import numpy as np
    import torch

    from paper_1905_09395_amd import stev, synth
    dev = torch.device("cuda:0")
    prec = stev.F64 if args.precision == "f64" else stev.F32
    dtype = torch.float64 if prec == stev.F64 else torch.float32
    T, P, Y = synth.make_cells_mech19(args.cells)
    ctx = stev.Context(0)
    ctx.set_stream(torch.cuda.current_stream(dev))
    gm = ctx.mechanism(synth.make_mech19())
    th = {"poly": stev.THERMO_POLY, "mlp": stev.THERMO_MLP, "ann": stev.THERMO_ANN}[args.thermo]
    if th == stev.THERMO_MLP:
        # a short schedule: the probe times the evaluation, not the fit (and a
        # counter-collecting profiler copes with fewer training dispatches)
        ctx.train_thermo_mlp(gm, epochs=20, n_samples=1 << 16, batch=8192, lr=3e-3, seed=104)
    if th == stev.THERMO_ANN:
        rep, prm = ctx.train_thermo_lma(gm, iters=150, n_samples=1 << 16, seed=104)
        ctx.set_thermo_ann(gm, rep["hidden"], 300.0, 3000.0, prm)

    def run(idx):
        Tt = torch.tensor(T[idx], dtype=dtype, device=dev)
        Pt = torch.tensor(P[idx], dtype=dtype, device=dev)
        Yt = torch.tensor(Y[idx], dtype=dtype, device=dev).contiguous()
        it = torch.zeros(len(idx), dtype=torch.int32, device=dev)
        st = ctx.integrate(gm, Tt, Pt, Yt, 1e-4,
                           params=stev.default_params(precision=prec, thermo=th,
                                                      stab_limit=1 if args.stab else 0),
                           iters=it)[1]
        return st, it.cpu().numpy()

    st_f, its = run(np.arange(len(T)))
    slow = int(np.argmax(its))
    st, it1 = run(np.array([slow]))
    n = int(it1[0])
    out = dict(cell=slow, iterations=n, solo_launch_ms=st["launch_ms"],
               us_per_iteration=1e3 * st["launch_ms"] / n, field_launch_ms=st_f["launch_ms"],
               field_over_solo=st_f["launch_ms"] / st["launch_ms"], precision=args.precision,
               thermo=args.thermo, stab_limit=bool(args.stab))
    ctx.close()
    return out


def run_legs(args):
    """The metric's other legs at reduced repetition, for the default line:
    batched, learned thermo (tanh and sigmoid networks against the
    polynomials) and served (p50 / p99 against plain per-request calls)."""
    import copy
    legs = {}
    la = copy.copy(args)
    la.steps, la.warmup = 2, 1
    b = run_batched(la)
    bc = b["config"]
    legs["batched"] = dict(cells_per_s=b["value"], ms_per_step=b["ms_per_step"],
                           plain_per_batch_cells_per_s=bc["plain_per_batch_cells_per_s"],
                           speedup_vs_plain_per_batch=bc["speedup_vs_plain_per_batch"],
                           network_cells_per_s=bc["batched_network_cells_per_s"],
                           network_speedup_vs_plain_per_batch=bc[
                               "batched_network_speedup_vs_plain_per_batch"],
                           rel_T_vs_fp64=bc["rel_T_vs_fp64"],
                           roofline_frac=b["roofline"]["frac"], workload=bc["workload"])
    print("legs: batched done", file=sys.stderr, flush=True)
    m = run_mlp(la)
    c = m["config"]
    legs["learned_thermo"] = dict(
        network_cells_per_s=m["value"], poly_cells_per_s=c["poly_cells_per_s"],
        sigmoid_cells_per_s=c["sigmoid_cells_per_s"],
        network_over_poly_time=c["network_over_poly_time"],
        sigmoid_over_poly_time=c["sigmoid_over_poly_time"],
        p99_rel_T=dict(network=c["network"]["p99_rel_T"],
                       sigmoid=c["sigmoid_network"]["p99_rel_T"],
                       poly=c["polynomials"]["p99_rel_T"]),
        accuracy_sample=c["accuracy_sample"], workload=c["workload"])
    print("legs: learned thermo done", file=sys.stderr, flush=True)
    ls = copy.copy(args)
    ls.steps, ls.warmup = 1, 1
    sv = run_serve(ls)
    legs["served"] = dict(loads=sv["config"]["loads"], hbm_budget_bytes=sv["config"]["hbm_budget_bytes"],
                          workload=sv["config"]["workload"])
    print("legs: served done", file=sys.stderr, flush=True)
    return legs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--cells", type=int, default=262144)
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--stab", action="store_true",
                    help="plain workload with the Eq 25 step cap (2/||A||_inf)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--solo", action="store_true",
                    help="the field's slowest cell integrated alone: per-iteration latency")
    ap.add_argument("--thermo", default="poly", choices=["poly", "mlp", "ann"],
                    help="--solo: thermo mode (mlp: FP32 only)")
    ap.add_argument("--no-legs", action="store_true",
                    help="plain workload only: skip the batched, learned-thermo and served legs")
    ap.add_argument("--probe", action="store_true",
                    help="counter-calibration run: one plain copy, then one step")
    ap.add_argument("--workload", default="plain",
                    choices=["plain", "batched", "mlp", "serve", "c3m"])
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="CPU only: write the HBM traffic summary from two counter runs")
    ap.add_argument("--pmc-summary", nargs="+", metavar="CSV",
                    help="CPU only: summarise counter runs of the integration launch")
    args = ap.parse_args()
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary, args.precision, args.cells)
        return
    if args.pmc_summary:
        pmc_summary(args.pmc_summary, args.precision, args.cells)
        return
    if args.probe:
        args.steps, args.warmup, args.no_cpu, args.no_legs = 1, 0, True, True
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (cells are independent; sharding them "
              "over several GPUs is described, not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1905_09395_amd import stev, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.solo:
        print(json.dumps(run_solo(args)), flush=True)
        return
    if args.workload != "plain":
        out = {"batched": run_batched, "mlp": run_mlp, "serve": run_serve,
               "c3m": run_c3m}[args.workload](args)
        print(json.dumps(out), flush=True)
        return
    dev = torch.device("cuda:0")
    if args.probe:
        traffic_probe(args.precision)
    mech = synth.make_mech19()
    T, P, Y = synth.make_cells_mech19(args.cells)
    dt = 1e-4
    prec = stev.F64 if args.precision == "f64" else stev.F32
    dtype = torch.float64 if prec == stev.F64 else torch.float32

    ctx = stev.Context(0)
    stream = torch.cuda.current_stream(dev)
    ctx.set_stream(stream)
    gm = ctx.mechanism(mech)
    T0 = torch.tensor(T, dtype=dtype, device=dev)
    P0 = torch.tensor(P, dtype=dtype, device=dev)
    Y0 = torch.tensor(Y, dtype=dtype, device=dev).contiguous()
    Tw, Yw = T0.clone(), Y0.clone()
    prm = stev.default_params(precision=prec, lanes_per_cell=args.lanes,
                              stab_limit=1 if args.stab else 0)

    def step():
        Tw.copy_(T0)
        Yw.copy_(Y0)
        return ctx.integrate(gm, Tw, P0, Yw, dt, params=prm)[1]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    kernel_ms, launch_ms, iters = [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = step()
        kernel_ms.append(st["kernel_ms"])
        launch_ms.append(st["launch_ms"])
        iters.append(st["total_iters"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0

    n = args.cells
    value = n * args.steps / el
    flops_pair, transc = gm.model_flops(stev.THERMO_POLY)
    flops_iter = direct_dft_flops(mech)
    # the dominant kernel is the persistent integration launch: its own
    # HIP-event time (the dispatch-order kernels and the probe before it are
    # part of the call's kernel_ms, not of this launch)
    k_ms = float(np.mean(launch_ms))
    work = float(np.mean(iters)) * flops_iter
    achieved = work / (k_ms * 1e-3) / 1e12
    peak = PEAK[args.precision]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": f"plain STEV, 19-species/50-reversible-reaction synthetic "
                               f"mechanism, {n} cells (70% 300-900 K, 30% 1400-2500 K), "
                               f"dt_flow=1e-4 s, {args.precision}" +
                               (", every step also capped at 2/||A||_inf (Eq 25)"
                                if args.stab else ""),
                   "cells": n, "dt_flow": dt, "lanes_per_cell": st["lanes_per_cell"],
                   "waves_per_wg": st["waves_per_wg"], "grid_wgs": st["grid_wgs"],
                   "cell_iterations_per_step": int(np.mean(iters)),
                   "max_cell_iterations": st["max_cell_iters"],
                   "call_kernel_ms": float(np.mean(kernel_ms)),
                   # Sec 2.4: cells still integrating at iteration i, at the
                   # histogram's bin edges where the load changes
                   "load_curve": stev.load_curve(st["load_hist"])},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     # the committed counters are those of the plain kernel in
                     # its default shape
                     "traffic": (None if args.stab or args.lanes
                                 else measured_traffic(args.precision, n)),
                     "kernel_ms": k_ms, "flop_count": "direct 13-point DFT",
                     "model_flop_per_cell_iter": flops_iter,
                     "flop_per_cell_iter_pair_symmetric_dft": flops_pair,
                     "frac_pair_symmetric_dft": float(np.mean(iters)) * flops_pair
                     / (k_ms * 1e-3) / 1e12 / peak,
                     "transcendentals_per_cell_iter": transc},
    }
    # end to end with host-resident (pinned) arrays: PCIe copies in and out
    # included; a side figure, never `value`
    if not args.probe:
        Th = torch.tensor(T, dtype=dtype).pin_memory()
        Ph = torch.tensor(P, dtype=dtype).pin_memory()
        Yh = torch.tensor(Y, dtype=dtype).contiguous().pin_memory()
        Th2, Yh2 = Th.clone().pin_memory(), Yh.clone().pin_memory()
        ctx.integrate(gm, Th2, Ph, Yh2, dt, params=prm)       # staging buffers
        e2e = []
        for _ in range(2):
            Th2.copy_(Th)
            Yh2.copy_(Yh)
            t1 = time.perf_counter()
            ctx.integrate(gm, Th2, Ph, Yh2, dt, params=prm)
            e2e.append(time.perf_counter() - t1)
        out["config"]["host_arrays_cells_per_s"] = n / min(e2e)
    if out["roofline"]["traffic"] is not None:
        # measured HBM bytes over this run's launch time, against the 8 TB/s peak
        out["roofline"]["traffic_gb_per_s"] = out["roofline"]["traffic"] / (k_ms * 1e-3) / 1e9
    cflops = None if args.stab or args.lanes else counted_flops(args.precision, n)
    if cflops is not None:
        # issued lane-slots, not algorithmic work: idle lanes and the software
        # exp/log/divide expansions count here, so this is no roofline fraction
        out["roofline"]["issued_valu_lane_tflops"] = cflops / (k_ms * 1e-3) / 1e12
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(mech, T, P, Y, dt)
    gm.close()
    ctx.close()
    if not args.no_legs:
        out["legs"] = run_legs(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
