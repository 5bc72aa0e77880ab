#!/usr/bin/env python3
"""Benchmark: exact amplitudes of a 6x6 (1+40+1) random circuit on one MI355X.

One step = one psim_amplitudes call on a batch of 16 bitstrings that share
rows 1-5 and differ in the last row (the whole hot path: every row of the
row scheme, every site contraction, rescaling, final assembly).  The value
is seconds per amplitude; the line also carries the contraction TFLOP/s
(8 real flops per complex multiply-add of the exact row-scheme count), the
hot kernel's roofline (interior-site contraction, eq. S4, timed with HIP
events on its launch stream), and the CPU oracle timed on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--prec fp32_3m|fp32|fp64|bf16x3] [--no-fp64] [--no-split-acc]
                    [--budget-s S]

Wall-clock budget: a 6x6 step takes tens of seconds, so the whole run is held
to --budget-s seconds from process start (default 440).  At most one warm-up
step runs when a step exceeds 10 s, and the timed loop stops early once the
remaining budget is needed for the legs that follow (FP64 path, single
amplitude, square partition, plain FP64 GPU, CPU oracle), each of which runs
one untimed-warmup-free step.  `steps` and `warmup` in the JSON line are the
steps that actually ran; every timed step is the full 16-bitstring batch.

The default path is the FP32-MFMA 3M scheme with partial sums in the K loops
(split accumulation): the FP32 form that meets the 1e-5 relative
bar on every oracle amplitude of this workload (without split accumulation
the worst is 1.25e-5).  The FP64 path is timed on the same batch for the
comparison the metric names.  --no-split-acc runs the FP32 forms with plain
sequential sums (faster, less accurate).
"""
import argparse
import hashlib
import json
import os
import sys
import time

T_START = time.monotonic()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "seconds/amplitude + contraction TFLOP/s (% MFMA peak), 6x6 d40, FP32-MFMA vs FP64"
# MI355X dense MFMA peaks (TFLOP/s) of the arithmetic each path issues
PEAK_TFLOPS = {"fp32": 157.3, "fp32_3m": 157.3, "fp64": 78.6, "bf16x3": 2500.0}
ISSUED_PER_CMAC = {"fp32": 8, "fp32_3m": 6, "fp64": 8, "bf16x3": 24}   # real MFMA flops per complex multiply-add
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_interior_site_6x6_d40_{prec}{split}.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Section of kernels.hip that holds each precision's hot kernel (between two
# "// ----...---- <name>" marker lines); traffic counters are tied to its hash.
KERNEL_SECTIONS = {"fp32_3m": ("3M, direct-to-LDS", "4M, direct-to-LDS"), "fp32": ("4M, direct-to-LDS", "BF16x3")}


def kernel_source_hash(prec):
    with open(os.path.join(ROOT, "paper_1905_08394_amd", "csrc", "kernels.hip")) as f:
        lines = f.read().split("\n")
    first, last = KERNEL_SECTIONS[prec]
    marker = "// " + "-" * 64 + " "
    a = lines.index(marker + first)
    b = lines.index(marker + last)
    return hashlib.sha256("\n".join(lines[a:b]).encode()).hexdigest()


def workload_base(lattice, seed=0):
    import rqcgen
    return rqcgen.bitstrings(lattice, lattice, seed, 1)[0]


def workload(lattice, depth, seed=0):
    import rqcgen
    c = rqcgen.generate(lattice, lattice, depth, seed)
    base = rqcgen.bitstrings(lattice, lattice, seed, 1)[0]
    cols = list(range(lattice - 4, lattice))
    return c, rqcgen.last_row_variants(base, lattice, lattice, cols)


def since_start():
    return time.monotonic() - T_START


def run_gpu(args, prec, circuit, bits, sweep=0, steps=None, warmup=None, reserve=None):
    """Plan, warm up and time `steps` full steps of the batch.  `reserve(t)`
    gives the seconds the legs after this one need when a step takes t
    seconds; the timed loop stops once another step would eat into them (at
    least one step always runs).  Returns the amplitudes, the timed seconds,
    the per-class profile, the plan stats and the (warmup, steps) that ran."""
    import torch
    import paper_1905_08394_amd as ps
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    peps = ps.Peps(circuit)
    plan = ps.Plan(peps, prec=prec, mem_budget=args.mem_gib << 30, max_batch=len(bits),
                   split_acc=args.split_acc and prec in ("fp32", "fp32_3m"), sweep=sweep)
    peps.close()
    stats = plan.stats()
    plan.workspace()                               # allocate before timing
    stream = torch.cuda.current_stream()
    if args.tune:
        t0 = time.perf_counter()
        best = plan.tune(reps=2)
        stats = plan.stats()
        log(f"tuned in {time.perf_counter() - t0:.1f}s: hot config {stats['hot_cfg']} ({best:.2f} ms per launch)")
    # prime the code objects with a tiny circuit (not a step)
    import rqcgen
    small = ps.Plan(ps.Peps(rqcgen.generate(3, 3, 8, 0)), prec=prec)
    small.amplitudes(rqcgen.bitstrings(3, 3, 0, 1))
    small.close()
    step_s = None
    ran_warmup = 0
    while ran_warmup < warmup:
        log(f"warmup {ran_warmup + 1}/{warmup} ({prec}) at {since_start():.0f}s")
        t0 = time.perf_counter()
        plan.amplitudes(bits, stream=stream.cuda_stream)
        torch.cuda.synchronize()
        step_s = time.perf_counter() - t0
        ran_warmup += 1
        if step_s > 10.0:                           # long steps: one warm-up is enough
            break
    plan.profile_start()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ran = 0
    while ran < steps:
        amps = plan.amplitudes(bits, stream=stream.cuda_stream)
        torch.cuda.synchronize()
        ran += 1
        el = time.perf_counter() - t0
        step_s = el / ran
        log(f"step {ran}/{steps} ({prec}) done at {el:.2f}s ({since_start():.0f}s since start)")
        if reserve is not None and ran < steps and \
                since_start() + step_s + reserve(step_s) > args.budget_s:
            log(f"budget: stopping the timed loop after {ran} of {steps} steps")
            break
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = plan.profile_read()
    plan.profile_stop()
    plan.close()
    return amps, elapsed, prof, stats, (ran_warmup, ran)


def golden_errors(bits, amps, lattice, depth):
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"rqc_{lattice}x{lattice}_d{depth}_s0.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    gb = np.array(g["bits"], dtype=np.uint8)
    ref = np.array(g["amps_re"]) + 1j * np.array(g["amps_im"])
    idx = [int(np.where((gb == b).all(axis=1))[0][0]) for b in bits]
    r = ref[idx]
    d = np.abs(amps - r)
    n = lattice * lattice
    # every amplitude's error, with x = 2^N |a_ref|^2 beside it (Porter-Thomas
    # tail amplitudes, x << 1, stay visible)
    return {"max_eps_rel": float(np.max(d / np.abs(r))), "median_eps_rel": float(np.median(d / np.abs(r))),
            "max_eps_rms": float(np.max(d) * 2 ** (n / 2)), "n": int(len(r)),
            "eps_rel": [float("%.3e" % v) for v in d / np.abs(r)],
            "x": [float("%.4g" % v) for v in np.abs(r) ** 2 * 2.0 ** n]}


def host_description():
    """Host CPU model, logical CPUs and numpy's BLAS, for the CPU timings."""
    import numpy as np
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = None
    try:
        cfg = np.show_config(mode="dicts")
        b = cfg.get("Build Dependencies", {}).get("blas", {})
        blas = f"{b.get('name')} {b.get('version')}".strip()
    except Exception:
        pass
    return {"cpu": model, "logical_cpus": os.cpu_count(), "blas": blas}


def cpu_baseline(circuit, bits, target_seconds):
    """The oracle's row scheme (numpy FP64) on (v, w) slices of one interior row."""
    import numpy as np
    from oracle import complexity as cx
    from oracle import peps as op
    L = circuit.lh
    P = op.build(circuit)
    dims = op.bond_dims(P)
    D = dims[("v", 1, 0)]
    sites = op.projected_sites(P, bits[0])
    rng = np.random.default_rng(0)
    labels = [("v", 1, c) for c in range(L - 1)]   # boundary after row 1, last leg fixed (v)
    shape = [dims[x] for x in labels]
    Fv = op.LT(rng.standard_normal(shape) + 1j * rng.standard_normal(shape), labels)
    row = 2
    # one (v, w) task: v = last input leg, w = first output leg; 1/D^2 of the row's work
    t0 = time.perf_counter()
    tasks = 0
    while True:
        op.row_transfer(Fv, sites, row, L, fixed={("v", 1, L - 1): tasks % D, ("v", 2, 0): tasks % D})
        tasks += 1
        if time.perf_counter() - t0 >= target_seconds:
            break
    t = time.perf_counter() - t0
    per_row = cx.row_scheme_cmac_per_row(L, L, dims)
    task_cmac = per_row[row] / (D * D)
    # batch: rows 0..L-2 once, the last row once per bitstring
    batch_cmac = sum(per_row[:-1]) + len(bits) * per_row[-1]
    s_per_amp = t / tasks * batch_cmac / task_cmac / len(bits)
    threads = int(os.environ.get("OPENBLAS_NUM_THREADS", os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    return {"value": s_per_amp, "unit": "s/amplitude", "cores": min(threads, os.cpu_count() or 1),
            "kind": "oracle", "host": host_description(),
            "sample": f"{tasks} (v,w) slice(s) of one interior row of the 6x6 (1+40+1) row scheme "
                      f"(oracle.peps.row_transfer, numpy complex128, {t:.1f} s), extrapolated by exact "
                      f"multiply-add counts to the 16-bitstring batch ({batch_cmac:.3e} CMAC)"}


def square_leg(args, circuit, bits, row_value):
    """The square partition on the batch the row scheme ran: seconds per
    amplitude, its exact multiply-add count, and the join GEMMs (the
    D^h x D^h x D^h steps, class 1 of the profile) against the MFMA peak."""
    a = argparse.Namespace(**vars(args))
    a.tune = False
    a.mem_gib = max(args.mem_gib, 64 if args.prec != "fp64" else 128)   # quadrant tensors of 8 GiB each
    log("square partition ...")
    amps, el, prof, stats, (_, ran) = run_gpu(a, args.prec, circuit, bits, sweep=3, steps=1, warmup=0)
    n_amp = ran * len(bits)
    issued = ISSUED_PER_CMAC[args.prec]
    cmac = sum(v["cmac"] for v in prof.values())
    j = prof["interior_site"]   # class 1 of a square plan: the joins
    join_tflops = issued * j["cmac"] / (j["ms"] / 1e3) / 1e12 if j["ms"] > 0 else None
    out = {"s_per_amplitude": el / n_amp, "speedup_vs_row_scheme": row_value / (el / n_amp),
           "cmac_per_step": cmac, "contraction_tflops": 8 * cmac / el / 1e12,
           "workspace_gib": round(stats["workspace_bytes"] / 2 ** 30, 2),
           "kernel_ms": {k: round(v["ms"], 3) for k, v in
                         zip(("quadrant_sites", "joins", "permute_pack_dot", "rescale"), prof.values())},
           "joins": {"achieved": join_tflops, "peak": PEAK_TFLOPS[args.prec], "unit": "TFLOP/s",
                     "frac": join_tflops / PEAK_TFLOPS[args.prec] if join_tflops else None,
                     "launches": j["launches"]}}
    err = golden_errors(bits, amps, args.lattice, args.depth)
    if err:
        out["vs_oracle"] = err
    return out


def single_leg(args, circuit, bits):
    """One amplitude on its own: the base bitstring of the batch in a
    psim_amplitudes call of one bitstring (no sharing), one step."""
    import numpy as np
    a = argparse.Namespace(**vars(args))
    base = bits[:1]
    for i, b in enumerate(bits):
        if np.array_equal(b, workload_base(args.lattice)):
            base = bits[i:i + 1]
    log("single amplitude ...")
    amps, el, prof, stats, (_, ran) = run_gpu(a, args.prec, circuit, base, steps=1, warmup=0)
    out = {"seconds": el / ran, "bitstrings": 1, "cmac": sum(v["cmac"] for v in prof.values()) / ran,
           "contraction_tflops": 8 * sum(v["cmac"] for v in prof.values()) / el / 1e12}
    err = golden_errors(base, amps, args.lattice, args.depth)
    if err:
        out["vs_oracle"] = err
    return out


def plain_fp64_gpu_baseline(stats, batch_cmac, nbits, reps=3):
    """The plain FP64 GPU contraction the target is compared with: the hot
    step (eq. S4) written the ordinary way, torch.tensordot on complex128
    (permute A to (m, u, l), then one complex GEMM in the vendor BLAS), at
    the 6x6 interior-row shape of one v slice (M = 32^4, K = N = 32^2).
    Timed with CUDA events on torch's stream; the batch total is extrapolated
    by the exact multiply-add count of the batch the library ran (the hot
    step carries 98 % of it)."""
    import torch
    torch.cuda.empty_cache()
    D = stats["chi"]
    L = stats["L"]
    M = D ** (L - 2)
    A = torch.randn(D, M, D, dtype=torch.complex128, device="cuda")   # [u][m][l]
    W = torch.randn(D, D, D * D, dtype=torch.complex128, device="cuda")  # [(u, l)][(d, r)]
    C = torch.tensordot(A, W, dims=([0, 2], [0, 1]))                    # warm
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        C = torch.tensordot(A, W, dims=([0, 2], [0, 1]))
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    step_cmac = M * D * D * D * D
    del A, W, C
    torch.cuda.empty_cache()
    return {"value": ms / 1e3 * batch_cmac / step_cmac / nbits, "unit": "s/amplitude",
            "kind": "torch complex128 tensordot (permute + vendor complex GEMM)",
            "step_ms": ms, "step_tflops": 8 * step_cmac / (ms / 1e3) / 1e12,
            "sample": f"{reps} interior-site steps of M = {M}, K = N = {D * D} complex128, extrapolated by "
                      f"exact multiply-add counts to the {nbits}-bitstring batch ({batch_cmac:.3e} CMAC)"}


def counters_program(prec="fp32_3m", reps=3, split_acc=False, tile_cfg=0):
    """Short program for rocprofv3 --pmc passes: a plain 4 GiB device copy (to
    calibrate FETCH_SIZE / WRITE_SIZE) and the interior-site contraction at the
    launch shape of the 6x6 (1+40+1) bench's interior sites before its rows
    were cut over w as well (two v values of M = 32^4, K = N = 32^2;
    complex64, complex128 for FP64), four times the work of one of its
    interior launches now."""
    import numpy as np
    import torch
    import paper_1905_08394_amd as ps
    n = 1 << 30                                   # 4 GiB of float32
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    M, K1, K2, N, batch = 32 ** 4, 32, 32, 1024, 2
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    eb = 16 if prec == "fp64" else 8
    A = torch.randn(batch * K1 * M * K2, dtype=dt, device="cuda")
    rng = np.random.default_rng(0)
    W = rng.standard_normal((K1 * K2, N)) + 1j * rng.standard_normal((K1 * K2, N))
    for r in range(reps):
        ps.contract_site(prec, A, W, M, K1, K2, N, batch=batch, split_acc=split_acc, tile_cfg=tile_cfg)
        log(f"hot step {r + 1}/{reps}")
    torch.cuda.synchronize()
    print(json.dumps({"prec": prec, "copy_bytes": 4 * n, "hot_step_algorithmic_bytes":
                      2 * batch * K1 * M * K2 * eb + K1 * K2 * N * eb // 2 * 4, "reps": reps}), flush=True)


def seven_program(args):
    """7x7 (1+40+1), the paper's flagship lattice (supplement S-IV), on one
    MI355X: built and planned exactly (host-only plan: the exact multiply-add
    count and the memory a one-GPU row sweep would need), then extrapolated
    from measured launches.  Its boundary F = 32^7 complex64 is 256 GiB, so two
    of them (input and output of a row) do not fit one GPU's 288 GB; nothing
    of the amplitude itself runs.  Timed: the interior-site contraction at the
    shape of a 7x7 row's (v, w) task -- the last input leg v and the first
    output leg w fixed: M = 32^4 rows, K = N = 1024, one task per launch, as
    the planner cuts a 7x7 row -- in the kernels the default precision runs
    (split accumulation, --tile-cfg), with synthetic operands (the kernel's
    speed does not depend on the values)."""
    import numpy as np
    import torch
    import paper_1905_08394_amd as ps
    import rqcgen
    torch.cuda.set_device(0)
    c = rqcgen.generate(7, 7, 40, 0)
    t0 = time.perf_counter()
    peps = ps.Peps(c)
    t_build = time.perf_counter() - t0
    plan = ps.Plan(peps, prec=args.prec, host_only=True, mem_budget=2 << 40, max_batch=1)
    st = plan.stats()
    plan.close()
    D, L = st["chi"], st["L"]
    # per-row multiply-adds of the row scheme on an L x L lattice with every
    # bond D (site shapes of eqs. S2-S6); their sum is checked against the plan
    first = sum(D ** (j + 3) for j in range(1, L - 1)) + D ** (L + 1)
    inner = 2 * D ** (L + 2) + (L - 2) * D ** (L + 3)
    last = D ** (L + 1) + sum(D ** (L - j + 2) for j in range(1, L - 1)) + D ** 2
    total = first + (L - 2) * inner + last
    assert abs(total / st["cmac_per_amplitude"] - 1) < 1e-12, (total, st["cmac_per_amplitude"])
    hot_cmac = (L - 2) * (L - 2) * D ** (L + 3)          # interior sites of interior rows (eq. S4)
    M, K1, K2, N, batch = D ** (L - 3), D, D, D * D, 1    # the plan cuts each 7x7 row into single (v, w) pairs
    split = args.split_acc and args.prec in ("fp32", "fp32_3m")
    A = torch.randn(batch * K1 * M * K2, dtype=torch.complex64, device="cuda")
    rng = np.random.default_rng(0)
    W = rng.standard_normal((K1 * K2, N)) + 1j * rng.standard_normal((K1 * K2, N))
    ps.contract_site(args.prec, A, W, M, K1, K2, N, batch=batch, split_acc=split, tile_cfg=args.tile_cfg)  # warm
    torch.cuda.synchronize()
    reps = 5
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        ps.contract_site(args.prec, A, W, M, K1, K2, N, batch=batch, split_acc=split, tile_cfg=args.tile_cfg)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps        # includes the per-call upload of W (8 MiB)
    rate = batch * M * K1 * K2 * N / (ms / 1e3)  # complex multiply-adds per second
    issued = ISSUED_PER_CMAC[args.prec]
    out = {"workload": "7x7 lattice, random circuit depth (1+40+1), D=32, one amplitude (row scheme)",
           "prec": args.prec, "split_accumulation": bool(split), "tile_cfg": args.tile_cfg, "peps_build_s": t_build, "cmac_per_amplitude": st["cmac_per_amplitude"],
           "cmac_per_row": {"first": first, "interior": inner, "last": last}, "hot_cmac_share": hot_cmac / total,
           "boundary_bytes": int(D ** L * 8), "one_gpu_row_sweep_workspace_bytes": st["workspace_bytes"],
           "hot_launch": {"shape": f"{batch} x (M = {M}, K = N = {K1 * K2})", "ms": ms,
                          "tflops_issued": issued * rate / 1e12, "frac_of_peak": issued * rate / 1e12 /
                          PEAK_TFLOPS[args.prec]},
           "extrapolated_s_per_amplitude": total / rate,
           "extrapolation": "exact multiply-add count of the amplitude / measured rate of the interior-site "
                            "contraction at the (v, w) task shape; boundary rows and rescales (about 2 % of "
                            "the work at 6x6) are counted at the same rate; the row sweep needs two 256 GiB "
                            "boundaries, more than one GPU holds, so this is a projection, not a run",
           "paper": "31 min per amplitude, 4096 Tianhe-2 fat nodes, FP64 (supplement S-IV)"}
    print(json.dumps(out), flush=True)


def fig2_program(args):
    """The paper's Fig. 2 experiment on our synthetic circuits: amplitudes of
    random bitstrings of an 8x8 (1+25+1) circuit (the paper used 10 000; the
    default here is 2048), the statistics of x = 2^N |a|^2
    against the Porter-Thomas law, and a histogram of ln x next to the
    log-transformed Porter-Thomas density exp(y - e^y)."""
    import numpy as np
    import torch
    import paper_1905_08394_amd as ps
    import rqcgen
    from oracle import stats
    n = args.fig2_count
    c = rqcgen.generate(8, 8, 25, 0)
    bits = rqcgen.bitstrings(8, 8, 7, n)
    peps = ps.Peps(c)
    chunk = 512
    plan = ps.Plan(peps, prec=args.prec, max_batch=chunk, mem_budget=args.mem_gib << 30, sweep=args.sweep)
    plan.workspace()
    plan.amplitudes(bits[:16])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    parts = []
    for s0 in range(0, n, chunk):
        parts.append(plan.amplitudes(bits[s0:s0 + chunk]))
        log(f"fig2 {args.prec}: {min(n, s0 + chunk)}/{n} amplitudes at {time.perf_counter() - t0:.1f}s")
    amps = np.concatenate(parts)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    x = stats.scaled_probabilities(amps, 64)
    summ = stats.porter_thomas_summary(x)
    edges = np.linspace(-8, 3, 23)
    hist, _ = np.histogram(np.log(x), bins=edges, density=True)
    mids = 0.5 * (edges[1:] + edges[:-1])
    print(json.dumps({"workload": f"8x8 (1+25+1), seed 0, {n} random bitstrings", "prec": args.prec,
                      "scheme": "square partition" if args.sweep == 3 else "row scheme",
                      "seconds": t, "s_per_amplitude": t / n, "cmac_per_amplitude": plan.stats()["cmac_per_amplitude"],
                      "porter_thomas": summ,
                      "log_histogram": [[round(float(m), 3), round(float(h), 4), round(float(stats.log_pt_density(m)), 4)]
                                        for m, h in zip(mids, hist)]}), flush=True)


def fast_sampling_program(args):
    """The fast-sampling reuse of the square partition (supplement S-II, the
    remark on sampling in one partition while the other regions' results are
    reused): 8x8 (1+25+1), one random bitstring and 4096 variants of it with
    random lower-right quadrants (16 qubits), against 4096 independent random
    bitstrings; seconds per amplitude of each."""
    import numpy as np
    import torch
    import paper_1905_08394_amd as ps
    import rqcgen
    torch.cuda.set_device(0)
    c = rqcgen.generate(8, 8, 25, 0)
    n = 4096
    base = rqcgen.bitstrings(8, 8, 3, 1)[0]
    lr = [r * 8 + col for r in range(4, 8) for col in range(4, 8)]
    fast = np.repeat(base[None, :], n, axis=0)
    fast[:, lr] = np.random.default_rng(5).integers(0, 2, size=(n, len(lr)), dtype=np.uint8)
    rand = rqcgen.bitstrings(8, 8, 7, n)
    plan = ps.Plan(ps.Peps(c), prec=args.prec, max_batch=512, mem_budget=(args.mem_gib or 64) << 30, sweep=3)
    plan.workspace()
    plan.amplitudes(rand[:16])
    out = {"workload": f"8x8 (1+25+1), seed 0, {n} bitstrings", "prec": args.prec, "scheme": "square partition"}
    for name, bits in (("lower_right_variants", fast), ("random", rand)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s0 in range(0, n, 512):
            plan.amplitudes(bits[s0:s0 + 512])
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        out[name] = {"seconds": t, "s_per_amplitude": t / n}
        log(f"fast sampling {name}: {t:.2f}s")
    out["speedup"] = out["random"]["seconds"] / out["lower_right_variants"]["seconds"]
    print(json.dumps(out), flush=True)


# Mixed batches: (lv, lh, depth) of circuits with uneven lattices and depths,
# seed = position in the list, a fixed number of random bitstrings each.
# "large": 3x3 .. 6x6 up to depth (1+24+1), 64 bitstrings each (the 6x6 d24
# circuit carries most of the work); "small": 48 circuits of at most 20
# qubits, 16 bitstrings each (launch-bound when run one by one).
MIXED = {
    "large": ([(3, 3, 8), (3, 4, 13), (2, 6, 16), (4, 4, 16), (4, 4, 24), (4, 5, 24),
               (5, 5, 16), (5, 5, 24), (3, 6, 24), (6, 6, 16), (5, 6, 24), (6, 6, 24)], 64),
    "small": ([(lv, lh, d) for d in (8, 12, 16, 20, 24, 13, 17, 21)
               for lv, lh in ((3, 3), (3, 4), (4, 4), (4, 5), (2, 6), (3, 5))], 16),
}


def mixed_program(args):
    """Mixed batches of circuits of uneven size and depth: every circuit's
    bitstrings contracted (a) plan by plan, one psim_amplitudes call each, and
    (b) all plans together in one psim_group_amplitudes call, whose merged
    launches cover the tiles of several circuits at once; each both eagerly
    and with HIP-graph replay."""
    import numpy as np
    import torch
    import paper_1905_08394_amd as ps
    import rqcgen
    for name, (spec, nbits) in MIXED.items():
        circuits, bits = [], []
        for k, (lv, lh, d) in enumerate(spec):
            circuits.append(rqcgen.generate(lv, lh, d, k))
            bits.append(rqcgen.bitstrings(lv, lh, k, nbits))
        res = {}
        times = {}
        merged = {}
        for graph in (False, True):
            plans = []
            for c, b in zip(circuits, bits):
                P = ps.Peps(c)
                plans.append(ps.Plan(P, prec=args.prec, max_batch=len(b), graph=graph))
                P.close()
            for p in plans:
                p.workspace()
            group = ps.Group(plans)
            cmac = sum(p.stats()["cmac_per_amplitude"] * len(b) for p, b in zip(plans, bits))
            tag = "_graph" if graph else ""
            fns = {"per_plan" + tag: lambda: [p.amplitudes(b) for p, b in zip(plans, bits)],
                   "grouped" + tag: lambda: group.amplitudes(bits)}
            for fname, fn in fns.items():
                res[fname] = fn()                       # warm (captures graphs)
                reps = max(args.steps, 7)
                l0 = group.stats()["grouped_launches"]
                ts = []
                for r in range(reps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    fn()
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                times[fname] = float(np.median(ts))
                merged[fname] = (group.stats()["grouped_launches"] - l0) // reps
                log(f"mixed {name} {fname}: median {times[fname] * 1e3:.2f} ms over {reps} runs")
            group.close()
            for p in plans:
                p.close()
        ref = res["per_plan"]
        same = all(all(np.array_equal(a, r) for a, r in zip(res[k], ref)) for k in res)
        n_amp = sum(len(b) for b in bits)
        best = min(times, key=times.get)
        print(json.dumps({
            "workload": f"mixed batch '{name}': " + ", ".join(f"{lv}x{lh} (1+{d}+1)" for lv, lh, d in spec) +
                        f"; {nbits} random bitstrings each, seeds 0..{len(spec) - 1}",
            "prec": args.prec, "circuits": len(spec), "amplitudes": n_amp, "cmac": cmac,
            "seconds": times, "speedup_grouped_vs_per_plan": times["per_plan"] / times["grouped"],
            "speedup_grouped_graph_vs_per_plan": times["per_plan"] / times["grouped_graph"],
            "best": best, "best_amplitudes_per_s": n_amp / times[best],
            "best_contraction_tflops": 8 * cmac / times[best] / 1e12,
            "merged_launches_per_call": merged["grouped"], "all_bitwise_equal_to_per_plan": same}), flush=True)


def measure_program(args):
    """Observables and sequential measurement through the double-layer
    network (psim_double_layer, psim_sample).  One double-layer PEPS with the
    slices (Z, I) at every site gives every product of Z's in one batched
    call: bitstring 0 at the sites the product covers, 1 elsewhere.
    Square partition, FP64 by default.  4x5 (1+16+1) (20 qubits): all <Z_q>,
    all nearest-neighbour <Z_a Z_b> and 512 sequential samples, against the
    oracle's state vector (timed beside it); 6x6 (1+16+1) (36 qubits, beyond a
    state vector): the same with 16 samples, checked by <psi|psi> = 1 and by
    p(bits) of every sample against |<bits|psi>|^2 from the ordinary
    amplitude path."""
    import numpy as np
    import torch
    import paper_1905_08394_amd as ps
    import rqcgen
    torch.cuda.set_device(0)
    Z = np.diag([1.0, -1.0]).astype(complex)
    prec = args.prec if args.prec != "bf16x3" else "fp64"

    def edges(lv, lh):
        return [(r * lh + c, r * lh + c + 1) for r in range(lv) for c in range(lh - 1)] + \
               [(r * lh + c, (r + 1) * lh + c) for r in range(lv - 1) for c in range(lh)]

    sweep = args.sweep or 3
    for lv, lh, d, S in ((4, 5, 16, 512), (6, 6, 16, 16)):
        c = rqcgen.generate(lv, lh, d, 0)
        n = lv * lh
        P = ps.Peps(c)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = np.zeros((n, 2, 2, 2), dtype=complex)
        o[:, 0] = Z
        o[:, 1] = np.eye(2)
        V = P.double_layer(o)
        E = edges(lv, lh)
        q = np.ones((1 + n + len(E), n), dtype=np.uint8)
        for k in range(n):
            q[1 + k, k] = 0
        for k, (a, b) in enumerate(E):
            q[1 + n + k, [a, b]] = 0
        plan = ps.Plan(V, prec=prec, max_batch=len(q), sweep=sweep)
        vals = plan.amplitudes(q)
        plan.close()
        torch.cuda.synchronize()
        t_obs = time.perf_counter() - t0
        norm = vals[0].real  # bitstring of all ones: identity everywhere
        zq, zz = vals[1:1 + n].real, vals[1 + n:].real
        u = np.random.default_rng(11).random((S, n))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bits, prob = ps.sample(P, u, prec=prec, sweep=sweep, max_batch=2 * S)
        torch.cuda.synchronize()
        t_smp = time.perf_counter() - t0
        out = {"workload": f"{lv}x{lh} (1+{d}+1), seed 0", "prec": prec, "scheme": "square partition" if sweep == 3
               else "row scheme", "double_layer_bond": int(V.info()["chi"]),
               "observables": {"count": len(q), "seconds": t_obs, "norm_minus_1": float(norm - 1)},
               "sampling": {"samples": S, "seconds": t_smp, "samples_per_s": S / t_smp,
                            "contractions": n, "bitstrings_per_contraction": 2 * S}}
        if n <= 20:
            from oracle import measure as om
            from oracle import statevector as sv
            t0 = time.perf_counter()
            psi = sv.run(c)
            ref_z = np.array([om.expectation(psi, {k: Z}).real for k in range(n)])
            ref_zz = np.array([om.expectation(psi, {a: Z, b: Z}).real for a, b in E])
            t_cpu_obs = time.perf_counter() - t0
            t0 = time.perf_counter()
            obits, oprob = om.sample_sequential(psi, u)
            t_cpu_smp = time.perf_counter() - t0
            out["vs_oracle"] = {"max_abs_err_z": float(np.max(np.abs(zq - ref_z))),
                                "max_abs_err_zz": float(np.max(np.abs(zz - ref_zz))),
                                "samples_identical": int(np.sum(np.all(bits == obits, axis=1))),
                                "max_rel_err_prob": float(np.max(np.abs(prob - oprob) / oprob)),
                                "cpu_seconds_observables": t_cpu_obs, "cpu_seconds_sampling": t_cpu_smp}
        else:
            amp = ps.Plan(P, prec="fp64", max_batch=S).amplitudes(bits)
            out["check"] = {"max_rel_err_prob_vs_amplitude_path": float(np.max(np.abs(prob - np.abs(amp) ** 2)
                                                                             / np.abs(amp) ** 2))}
        out["mean_z"] = float(np.mean(zq))
        print(json.dumps(out), flush=True)


def small_configs_program(args):
    """The smaller lattices of the parity suite timed through the library:
    3x3 (1+8+1) all 512 amplitudes, 4x5 (1+24+1) 64 random bitstrings for each
    of seeds 0-7 (eight plans, one grouped call), 5x5 (1+32+1) 256 random
    bitstrings in one call; median over repeats, graph replay on."""
    import numpy as np
    import torch
    import paper_1905_08394_amd as ps
    import rqcgen
    rows = []

    def timeit(fn, reps):
        fn()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    c = rqcgen.generate(3, 3, 8, 0)
    bits = rqcgen.all_bitstrings(9)
    pl = ps.Plan(ps.Peps(c), prec=args.prec, max_batch=len(bits), graph=True)
    t = timeit(lambda: pl.amplitudes(bits), 20)
    rows.append(("3x3 (1+8+1), all 512 amplitudes", len(bits), pl.stats()["cmac_per_amplitude"] * len(bits), t))
    plans, bl = [], []
    for seed in range(8):
        c = rqcgen.generate(4, 5, 24, seed)
        bl.append(rqcgen.bitstrings(4, 5, seed, 64))
        plans.append(ps.Plan(ps.Peps(c), prec=args.prec, max_batch=64, graph=True))
    g = ps.Group(plans)
    t = timeit(lambda: g.amplitudes(bl), 20)
    rows.append(("4x5 (1+24+1), seeds 0-7 x 64 random bitstrings (one grouped call)", 512,
                 sum(p.stats()["cmac_per_amplitude"] * 64 for p in plans), t))
    c = rqcgen.generate(5, 5, 32, 0)
    bits = rqcgen.bitstrings(5, 5, 0, 256)
    pl = ps.Plan(ps.Peps(c), prec=args.prec, max_batch=256, graph=True)
    t = timeit(lambda: pl.amplitudes(bits), 5)
    rows.append(("5x5 (1+32+1), 256 random bitstrings in one call", 256, pl.stats()["cmac_per_amplitude"] * 256, t))
    if args.prec != "bf16x3":
        sq = ps.Plan(ps.Peps(c), prec=args.prec, max_batch=256, sweep=3)
        t = timeit(lambda: sq.amplitudes(bits), 5)
        rows.append(("5x5 (1+32+1), 256 random bitstrings, square partition (eqs. S11-S12)", 256,
                     sq.stats()["cmac_per_amplitude"] * 256, t))
    cpu = small_configs_oracle_times() if not args.no_cpu_baseline else {}
    for name, n, cmac, t in rows:
        rec = {"workload": name, "prec": args.prec, "amplitudes": n, "seconds": t,
               "amplitudes_per_s": n / t, "cmac": cmac, "contraction_tflops": 8 * cmac / t / 1e12}
        key = name.split(",")[0]
        if key in cpu and "square" not in name:
            rec["cpu_oracle"] = cpu[key]
        print(json.dumps(rec), flush=True)
        log(f"{name}: {t * 1e3:.2f} ms")


def small_configs_oracle_times():
    """The oracle on the same small workloads (numpy FP64 on the host): all
    threads and one thread.  3x3 and 4x5: the state vector (all 512
    amplitudes; 8 seeds x 64 bitstrings); 5x5: the oracle's PEPS row scheme
    on a few of the 256 bitstrings plus its builder, extrapolated by count."""
    from threadpoolctl import threadpool_limits
    import rqcgen
    from oracle import peps as op
    from oracle import statevector as sv

    def sv_job(cases):
        for c, bits in cases:
            sv.amplitudes(sv.run(c), bits)

    c3 = [(rqcgen.generate(3, 3, 8, 0), rqcgen.all_bitstrings(9))]
    c45 = [(rqcgen.generate(4, 5, 24, s), rqcgen.bitstrings(4, 5, s, 64)) for s in range(8)]
    c5 = rqcgen.generate(5, 5, 32, 0)
    b5 = rqcgen.bitstrings(5, 5, 0, 256)
    out = {}
    for threads in (None, 1):
        with threadpool_limits(limits=threads):
            t0 = time.perf_counter()
            sv_job(c3)
            t3 = time.perf_counter() - t0
            t0 = time.perf_counter()
            sv_job(c45)
            t45 = time.perf_counter() - t0
            t0 = time.perf_counter()
            P = op.build(c5)
            tb = time.perf_counter() - t0
            k = 2 if threads is None else 1
            t0 = time.perf_counter()
            op.amplitudes(P, b5[:k])
            t5 = tb + (time.perf_counter() - t0) * 256 / k
        tag = "seconds" if threads is None else "seconds_1_thread"
        for key, v in (("3x3 (1+8+1)", t3), ("4x5 (1+24+1)", t45), ("5x5 (1+32+1)", t5)):
            threads_all = int(os.environ.get("OPENBLAS_NUM_THREADS", os.environ.get("OMP_NUM_THREADS", os.cpu_count())))
            out.setdefault(key, {"kind": "oracle", "threads": min(threads_all, os.cpu_count() or 1)})[tag] = v
    out["5x5 (1+32+1)"]["sample"] = "PEPS row scheme on 2 (1 thread: 1) of the 256 bitstrings, extrapolated"
    log(f"cpu oracle: {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--prec", default="fp32_3m", choices=["fp32", "fp32_3m", "fp64", "bf16x3"])
    ap.add_argument("--lattice", type=int, default=6,
                    help="6: the headline workload; 7: the 7x7 (1+40+1) projection from measured launches")
    ap.add_argument("--depth", type=int, default=40)
    ap.add_argument("--mem-gib", type=int, default=0, help="workspace budget (0: 32 GiB fp32, 48 GiB fp64)")
    ap.add_argument("--no-fp64", dest="compare_fp64", action="store_false",
                    help="skip timing the FP64 path on the same batch")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--budget-s", type=float, default=440.0,
                    help="wall-clock budget of the whole run, from process start")
    ap.add_argument("--no-single", dest="single", action="store_false",
                    help="skip timing one amplitude on its own")
    ap.add_argument("--no-tune", dest="tune", action="store_false", help="skip the tile autotuner")
    ap.add_argument("--no-split-acc", dest="split_acc", action="store_false",
                    help="FP32 4M / 3M with plain sequential K-loop sums instead of per-stage partial sums")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-square", dest="square", action="store_false",
                    help="skip timing the square partition on the same batch")
    ap.add_argument("--square-only", action="store_true",
                    help="only the square partition on the 6x6 batch (for profiling)")
    ap.add_argument("--counters", action="store_true", help="short program for rocprofv3 --pmc passes")
    ap.add_argument("--tile-cfg", type=int, default=0, help="--counters / --lattice 7: tile candidate of the launch")
    ap.add_argument("--fig2", action="store_true", help="8x8 (1+25+1) Porter-Thomas experiment")
    ap.add_argument("--fig2-count", type=int, default=2048)
    ap.add_argument("--sweep", type=int, default=0, help="--fig2: 0 row scheme, 3 square partition")
    ap.add_argument("--mixed", action="store_true", help="mixed batches of 3x3..6x6 circuits, grouped vs per plan")
    ap.add_argument("--small-configs", action="store_true", help="3x3, 4x5 and 5x5 parity workloads, timed")
    ap.add_argument("--fast-sampling", action="store_true",
                    help="square partition: bitstrings differing in one quadrant vs random ones (8x8 (1+25+1))")
    ap.add_argument("--measure", action="store_true",
                    help="observables and sequential measurement through the double-layer network")
    args = ap.parse_args()
    if args.fast_sampling:
        fast_sampling_program(args)
        return
    if args.measure:
        args.prec = "fp64" if args.prec == "fp32_3m" and "--prec" not in sys.argv else args.prec
        measure_program(args)
        return
    if args.small_configs:
        small_configs_program(args)
        return
    if args.mixed:
        mixed_program(args)
        return
    if args.fig2:
        args.mem_gib = args.mem_gib or 64
        fig2_program(args)
        return
    if args.lattice == 7:
        seven_program(args)
        return
    if args.counters:
        counters_program(args.prec, split_acc=args.split_acc and args.prec in ("fp32", "fp32_3m"),
                         tile_cfg=args.tile_cfg)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1).",
              file=sys.stderr)
        sys.exit(2)
    if args.mem_gib == 0:
        # the batch shares rows 1-5, so one boundary per row suffices: the plan
        # cuts the rows over v and w and needs 24 GiB (FP32) / 40 GiB (FP64)
        args.mem_gib = 48 if args.prec == "fp64" else 32

    import torch
    torch.cuda.set_device(0)
    circuit, bits = workload(args.lattice, args.depth)
    if args.square_only:
        print(json.dumps({"workload": f"{args.lattice}x{args.lattice} (1+{args.depth}+1), {len(bits)} bitstrings",
                          "prec": args.prec, "square_partition": square_leg(args, circuit, bits, float("nan"))}),
              flush=True)
        return
    log(f"workload {args.lattice}x{args.lattice} (1+{args.depth}+1), {len(bits)} bitstrings, {args.prec}")
    compare64 = args.compare_fp64 and args.prec != "fp64"
    cpu_on = not args.no_cpu_baseline
    square_on = args.square and args.lattice % 2 == 0 and args.prec in ("fp32", "fp32_3m", "fp64")

    def reserve(t):
        """Seconds the legs after the timed loop need when a step takes t s
        (FP64 steps take about 2.6 t, the square partition about 0.25 t)."""
        r = 15.0
        if compare64:
            r += 2.8 * t + 30.0 + 10.0                 # FP64 path (plan, upload, 1 step) + plain FP64
        if args.single:
            r += 1.05 * t + 10.0
        if square_on:
            r += 0.4 * t + 20.0
        if cpu_on:
            r += args.cpu_seconds + 15.0
        return r

    amps, elapsed, prof, stats, (ran_warmup, ran_steps) = run_gpu(args, args.prec, circuit, bits, reserve=reserve)
    step_s = elapsed / ran_steps
    n_amp = ran_steps * len(bits)
    cmac = sum(v["cmac"] for v in prof.values())
    tflops = 8 * cmac / elapsed / 1e12
    hot = prof["interior_site"]
    issued = ISSUED_PER_CMAC[args.prec]
    hot_tflops = issued * hot["cmac"] / (hot["ms"] / 1e3) / 1e12 if hot["ms"] > 0 else None
    peak = PEAK_TFLOPS[args.prec]
    traffic = None
    tr = None
    split_on = bool(args.split_acc and args.prec in ("fp32", "fp32_3m"))
    tfile = TRAFFIC_FILE.format(prec=args.prec, split="_split" if split_on else "")
    if os.path.exists(tfile) and args.lattice == 6:
        with open(tfile) as f:
            tr = json.load(f)
    per_launch_cmac = hot["cmac"] / max(hot["launches"], 1)
    # counters of this precision's hot kernel, while its source section is unchanged
    if tr is not None and args.prec in KERNEL_SECTIONS and tr.get("kernel_source_sha256") == kernel_source_hash(args.prec) \
            and "issued_flops_per_launch" in tr:
        # counters were taken on the largest interior launch; scale to this
        # run's average launch by issued flops (same K and N, M differs)
        traffic = tr["bytes_per_launch"] * issued * per_launch_cmac / tr["issued_flops_per_launch"]
    out = {
        "metric": METRIC,
        "value": elapsed / n_amp,
        "unit": "s/amplitude",
        "n_gpus": 1,
        "steps": ran_steps,
        "warmup": ran_warmup,
        "ms_per_step": elapsed / ran_steps * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        # the paper's own timings (FP64, CPUs; no 6x6 figure is published): context only
        "paper_context": {"7x7 (1+40+1)": "31 min per amplitude, 4096 Tianhe-2 fat nodes, FP64",
                          "7x7 (1+39+1)": "9 min per amplitude, 4096 Tianhe-2 nodes, FP64",
                          "8x8 (1+25+1)": "under 1 h per amplitude, 2-core 2.8 GHz PC"},
        "dtype": {"fp64": "f64", "bf16x3": "bf16x3"}.get(args.prec, "f32"),
        "data": "synthetic",
        "split_accumulation": split_on,
        "config": {"workload": f"{args.lattice}x{args.lattice} lattice, random circuit depth (1+{args.depth}+1), "
                               f"D={stats['chi']}, exact row-scheme amplitudes of {len(bits)} bitstrings "
                               f"sharing rows 1-{args.lattice - 1} (last-row variants)",
                   "precision": {"fp32": "complex64 storage, FP32 MFMA (4M)",
                                 "fp32_3m": "complex64 storage, FP32 MFMA (3M, Gauss)" +
                                            (", split K accumulation (partial sums)" if split_on else ""),
                                 "fp64": "complex128 storage, FP64 MFMA",
                                 "bf16x3": "complex64 storage, BF16 hi/lo split, 3 BF16 MFMA products, "
                                           "FP32 accumulation"}[args.prec],
                   "bitstrings_per_step": len(bits), "seed": 0, "v_chunk": stats["v_chunk"],
                   "w_chunk": stats["w_chunk"],
                   "hot_tile_config": stats["hot_cfg"],
                   "workspace_gib": round(stats["workspace_bytes"] / 2 ** 30, 2)},
        "contraction_tflops": tflops,
        "pct_mfma_peak": tflops / peak * issued / 8,
        "s_per_step_of_16": step_s,
        "budget": {"budget_s": args.budget_s, "requested_steps": args.steps, "requested_warmup": args.warmup},
        "kernel_ms": {k: round(v["ms"], 3) for k, v in prof.items()},
        # memory-bound classes: algorithmic bytes / their time, against 8 TB/s
        "hbm_kernels": {k: {"gb_per_s": round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1),
                            "frac_of_8tbs": round(v["bytes"] / (v["ms"] / 1e3) / 8e12, 3)}
                        for k, v in prof.items() if k != "interior_site" and v["ms"] > 0},
        "roofline": {
            "bound": "mfma", "achieved": hot_tflops, "peak": peak, "unit": "TFLOP/s",
            "frac": (hot_tflops / peak) if hot_tflops else None,
            "traffic": traffic,
            "kernel": "site_gemm (interior site, eq. S4)",
            "flops_per_launch": issued * per_launch_cmac, "launches": hot["launches"],
            "flops_counted": f"{issued} real MFMA flops issued per complex multiply-add",
            "avg_launch_ms": hot["ms"] / max(hot["launches"], 1),
        },
    }
    err = golden_errors(bits, amps, args.lattice, args.depth)
    if err:
        out["vs_oracle"] = err
    skipped = []

    def fits(seconds, name):
        if since_start() + seconds <= args.budget_s:
            return True
        skipped.append(name)
        log(f"budget: skipping {name} ({since_start():.0f}s used of {args.budget_s:.0f}s)")
        return False

    if compare64 and fits(2.8 * step_s + 30.0, "fp64"):
        a64 = argparse.Namespace(**vars(args))
        a64.mem_gib = 48
        a64.tune = False
        amps64, el64, prof64, _, (_, ran64) = run_gpu(a64, "fp64", circuit, bits, steps=1, warmup=0)
        h64 = prof64["interior_site"]
        out["fp64"] = {"s_per_amplitude": el64 / (ran64 * len(bits)),
                       "speedup_over_fp64": (el64 / ran64) / step_s, "steps": ran64, "warmup": 0,
                       "contraction_tflops": 8 * sum(v["cmac"] for v in prof64.values()) / el64 / 1e12,
                       "hot_kernel_tflops": 8 * h64["cmac"] / (h64["ms"] / 1e3) / 1e12,
                       "pct_fp64_mfma_peak": 8 * sum(v["cmac"] for v in prof64.values()) / el64 / 1e12 / 78.6}
        e64 = golden_errors(bits, amps64, args.lattice, args.depth)
        if e64:
            out["fp64"]["vs_oracle"] = e64
        import numpy as np
        d = np.abs(amps - amps64)
        out["vs_fp64_gpu"] = {"max_rel": float(np.max(d / np.abs(amps64))),
                              "median_rel": float(np.median(d / np.abs(amps64)))}
    if compare64 and args.lattice == 6 and fits(10.0, "plain_fp64_gpu"):
        log("plain FP64 GPU baseline (torch complex128) ...")
        out["plain_fp64_gpu"] = plain_fp64_gpu_baseline(stats, cmac / ran_steps, len(bits))
        out["vs_plain_fp64_gpu"] = out["plain_fp64_gpu"]["value"] / out["value"]
    if args.single and fits(1.05 * step_s + 10.0, "single_amplitude"):
        out["single_amplitude"] = single_leg(args, circuit, bits)
    if square_on and fits(0.4 * step_s + 20.0, "square_partition"):
        # the paper's square partition (Fig. S2(b), eqs. S9-S10) on the same batch
        out["square_partition"] = square_leg(args, circuit, bits, out["value"])
    if cpu_on and fits(args.cpu_seconds + 10.0, "cpu_baseline"):
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(circuit, bits, args.cpu_seconds)
    out["budget"]["skipped"] = skipped
    out["budget"]["wall_s_at_print"] = round(since_start(), 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
