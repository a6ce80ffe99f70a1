"""Benchmark of the frame-potential hot path on one MI355X.

Workload: local random circuits on n = 50 qubits (one Haar U(4) gate per step
on a uniformly chosen bond), S steps per circuit, 10^4 (U, V) pairs per
batch, complex64 with float64 scales and reduction.  One step = the whole
path over one batch: sample the gates, plan every pair on the device,
contract Tr(U^dagger V) for every pair, reduce F^(k), k = 1..3 (the reduction
returns the estimates to the host, which ends the step).  Three batches are
in flight on three streams: sampling runs two batches ahead, and a batch is
planned while the previous one is swept (serial_ms_per_step reports the same
steps one at a time).  The headline run has no per-launch HIP events (they cost time of
their own); kernel durations, the roofline and the step breakdown come from
runs with events (ms_per_step_with_events, serial_ms_per_step).  Inputs are
synthetic and seeded.

Prints one JSON line.  --gpus N with N > 1 exits: the library runs on one GPU
(how the work would shard across GPUs is a design, not code).
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Tr(U†V) contractions/s at n=50; time-to-1%-rel-err F^(2), CV vs plain"
PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector, published
PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector, published
PEAK_HBM_GBS = 8000.0
SWEEP_CLASSES = ("lds16", "lds64", "lds256", "lds1024", "hbm", "hea")
# sweep rate assumed when a deep batch is planned: batches at 300 and 350
# steps ran their sweeps at 1.4-3.5 TFLOP/s (pairs of 2^34 entries
# included); the cap assumes 0.5
DEEP_PLAN_TFLOPS = 0.5
# kernel of each sweep class for local random batches (names as rocprofv3 shows them)
LR_KERNELS = {
    "lds16": "fp::sweep_wave_kernel<{r}, 8, 4, false>", "lds64": "fp::sweep_wave_kernel<{r}, 10, 2, false>",
    "lds256": "fp::sweep_lds_kernel<{r}, 256, 1, false>", "lds1024": "fp::sweep_lds_kernel<{r}, {big}, 1, false>",
    "hbm": "fp::sweep_hbm_kernel<{r}, 512, false, int, false>"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50, help="batches timed in each headline run")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--depth", type=int, default=100, help="steps per circuit of the headline workload")
    ap.add_argument("--pairs", type=int, default=10000)
    ap.add_argument("--n", type=int, default=50)
    ap.add_argument("--in-flight", type=int, default=3, help="batches in flight (buffers and streams) in the timed runs")
    ap.add_argument("--precision", default="c64", choices=["c64", "c128"])
    ap.add_argument("--depth-steps", type=int, default=6, help="batches timed per step count of --per-depth")
    ap.add_argument("--per-depth", default="50,100,150,200,250,300",
                    help="comma list of step counts measured besides the headline ('' = none)")
    ap.add_argument("--deep-depths", default="350",
                    help="comma list of step counts past --per-depth, timed on smaller batches one at a time "
                         "('' = none; skipped too with --per-depth '')")
    ap.add_argument("--deep-pairs", type=int, default=1000, help="pairs per batch of --deep-depths")
    ap.add_argument("--deep-batches", type=int, default=2, help="batches timed per step count of --deep-depths")
    ap.add_argument("--deep-cap-s", type=float, default=60.0,
                    help="a --deep-depths batch whose planned sweep work would take longer than this at "
                         "DEEP_PLAN_TFLOPS is reported with its plan and not run")
    ap.add_argument("--feasibility", default=",".join(str(x) for x in range(50, 801, 50)),
                    help="comma list of step counts whose register widths are reported ('' = none)")
    ap.add_argument("--feasibility-pairs", type=int, default=0,
                    help="pairs sampled per step count (0: a whole batch up to 400 steps, 2000 beyond)")
    ap.add_argument("--cpu-seconds", type=float, default=8.0, help="length of each of the three oracle windows")
    ap.add_argument("--out", default="", help="also write the full record (per step count, ensembles, "
                                             "control variate) to this JSON file")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cv", action="store_true", help="skip the control-variate experiment (HEA n=40, L=6)")
    ap.add_argument("--no-suite", action="store_true", help="skip the other ensembles (brickwork n=6, n=20; HEA n=30)")
    ap.add_argument("--suite-pairs", type=int, default=100000)
    ap.add_argument("--cv-surrogate", type=int, default=1000000)
    ap.add_argument("--serial", action="store_true",
                    help="time one batch at a time only (the profiling runs use it so that their kernel "
                         "durations are those the roofline divides by)")
    ap.add_argument("--layer-scaling-n", default="",
                    help="comma list of n: layers to an epsilon = 0.1 design of brickworks per n and their slope "
                         "in n (not run by default)")
    ap.add_argument("--layer-scaling-pairs", type=int, default=20000)
    ap.add_argument("--layer-scaling-ansatz", default="brickwork", choices=["brickwork", "pauli_cnot"])
    ap.add_argument("--with-copy", action="store_true",
                    help="also run one 256 MiB device copy (counter calibration for PMC runs)")
    return ap.parse_args()


_STREAMS = []


def bench_streams(torch, k):
    """The first k of the streams every run uses: created once, together and
    before the library creates its side streams, straight through the HIP
    runtime (torch's stream pool hands out streams that already share the
    process's four hardware queues), so that each batch in flight has a
    hardware queue of its own."""
    import ctypes
    try:
        hip = ctypes.CDLL("libamdhip64.so.7")  # the runtime torch has loaded
    except OSError:
        hip = None  # another runtime name: torch's own streams (slower queue layout)
    while len(_STREAMS) < k:
        h = ctypes.c_void_p()
        if hip is None:
            _STREAMS.append(torch.cuda.Stream())
            continue
        if hip.hipStreamCreateWithFlags(ctypes.byref(h), 1) != 0:  # hipStreamNonBlocking
            raise RuntimeError("hipStreamCreateWithFlags failed")
        _STREAMS.append(torch.cuda.ExternalStream(h.value))
    return _STREAMS[:k]


def progress(msg):
    """One line per finished stage on stderr (stdout carries only the JSON line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def run_workload(fp, torch, n, depth, pairs, prec, steps, warmup, seed_base, pipeline=True, in_flight=2,
                 profile=True, say_batches=False):
    """Times `steps` batches.  Pipelined: `in_flight` buffers (gates, traces,
    workspace) on streams of their own.  Sampling runs in_flight - 1 batches
    ahead of contraction: batch i + in_flight - 1 is sampled as soon as batch
    i - 1's reduction has returned (its buffer is then free), so that while
    the host waits for batch i's plans (the contraction reads the planner's
    register widths back), the device runs batch i - 1's sweeps, batch i's
    planner and the next samplers side by side.  Every batch is sampled,
    contracted and reduced exactly once inside the timed region.  One at a
    time, `say_batches` prints a line as each batch ends."""
    ens = fp.Ensemble(fp.LOCAL_RANDOM, n, depth)
    nbuf = in_flight if pipeline else 1
    gates = [fp.alloc_gates(ens, pairs, prec) for _ in range(nbuf)]
    trace = [torch.empty(2 * pairs, dtype=torch.float64, device="cuda") for _ in range(nbuf)]
    wsb = fp.fp_workspace_bytes(ens, pairs, prec)
    ws = [torch.empty(wsb, dtype=torch.uint8, device="cuda") for _ in range(nbuf)]
    streams = bench_streams(torch, nbuf)
    seed = seed_base | (depth << 32)

    def sample(i):
        b = i % nbuf
        fp.fp_sample_gates(ens, pairs, seed, i * pairs, prec, gates[b], streams[b])

    def contract(i):
        b = i % nbuf
        fp.fp_contract_trace_batch(ens, pairs, prec, gates[b], trace[b], ws[b], streams[b])

    def finish(i):
        b = i % nbuf
        return fp.fp_frame_potential(trace[b], pairs, 3, streams[b])

    def run(first, count):
        f = None
        end = first + count
        if count <= 0:
            return f
        if pipeline and nbuf > 1:
            for i in range(first, min(end, first + nbuf - 1)):
                sample(i)
            for i in range(first, end):
                contract(i)
                if i > first:
                    f = finish(i - 1)
                if i + nbuf - 1 < end:
                    sample(i + nbuf - 1)
            f = finish(end - 1)
        else:
            for i in range(first, end):
                sample(i)
                contract(i)
                f = finish(i)
                f_batches.append(f[0])
                if say_batches:
                    progress(f"S={depth}: batch {i + 1} of {end} done")
        return f

    f_batches = []

    run(0, warmup)
    torch.cuda.synchronize()
    f_batches.clear()
    if profile:  # HIP events around every launch (they cost time of their own)
        fp.fp_profile_begin()
    t0 = time.perf_counter()
    f = run(warmup, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = fp.fp_profile_end() if profile else None
    progress(f"S={depth}: {steps} batches, {'pipelined' if pipeline else 'one at a time'}"
             f"{' with events' if profile else ''}: {wall / steps * 1e3:.3f} ms per batch")
    return {"wall_s": wall, "prof": prof, "F": f[0], "SE": f[1], "ws_bytes": wsb, "F_batches": f_batches}


def layer_scaling(fp, torch, traces_by_depth, n, k_max=3, resamples=300, epsilon=0.1):
    """The paper's uncertainty analysis and fit on the device: bootstrap of
    F^(k) at every depth (300 resamples), then per resample the exponential
    fit over the depths with (F - F_Haar)/F_Haar < 5 and the layers to an
    epsilon-approximate k-design; median and failed resamples per k."""
    depths = sorted(traces_by_depth)
    samples = torch.empty(len(depths), k_max, resamples, dtype=torch.float64, device="cuda")
    boot = {}
    for j, d in enumerate(depths):
        tr = traces_by_depth[d]
        med, lo, hi = fp.fp_bootstrap(tr, tr.numel() // 2, k_max, resamples, 0xB0075 + d, samples[j])
        boot[str(d)] = {"median": med, "lo95": lo, "hi95": hi}
    out = {"depths": depths, "bootstrap": boot, "layers_to_epsilon": {}}
    for k in range(2, k_max + 1):  # F^(1) equals its Haar value exactly for these ensembles: nothing to fit
        fk = samples[:, k - 1, :].contiguous()
        med, failed = fp.fp_layers_to_epsilon(fk, depths, resamples, fp.fp_haar_frame_potential(k, 2.0 ** n),
                                              epsilon, n, 2, k)
        out["layers_to_epsilon"][str(k)] = {"median": med, "failed_resamples": failed}
    return out


def layer_scaling_vs_n(fp, torch, np, synth, ns, pairs, ansatz=None, depths=None):
    """Layers to an epsilon = 0.1 approximate k-design for every n of `ns`
    (complex64, `pairs` pairs per depth, the same bootstrap and fit as
    layer_scaling), and the least-squares slope of those layers in n per k.
    Brickworks (the paper's parallel random unitaries, depths 2..10; the paper
    reports a slope of 4.38 for k = 2 from its own runs, context, not a
    target) or the paper's hardware-efficient ansatz with CNOT walls (layers
    2..7, the register of 2L - 1 bits in LDS)."""
    ansatz = fp.BRICKWORK if ansatz is None else ansatz
    if depths is None:
        depths = range(2, 11) if ansatz == fp.BRICKWORK else range(2, 8)
    per_n = {}
    for n in ns:
        traces = {}
        for d in depths:
            _, tr = fixed_topology(fp, torch, ansatz, n, d, pairs, fp.C64, synth.workload_seed(20 + 40 * ansatz + n, d),
                                   steps=1, chunk=min(pairs, 20000))
            traces[d] = tr
        per_n[str(n)] = layer_scaling(fp, torch, traces, n)["layers_to_epsilon"]
        progress(f"layer scaling n={n}: { {k: round(v['median'], 2) for k, v in per_n[str(n)].items()} }")
    slopes = {}
    for k in ("2", "3"):
        pts = [(int(n), v[k]["median"]) for n, v in per_n.items() if math.isfinite(v[k]["median"])]
        if len(pts) >= 2:
            x, y = np.array(pts, dtype=np.float64).T
            slope, icept = np.polyfit(x, y, 1)
            slopes[k] = {"slope": float(slope), "intercept": float(icept), "points": len(pts)}
    return {"ansatz": ansatz, "pairs_per_depth": pairs, "depths": list(depths), "layers_to_epsilon": per_n,
            "slope_in_n": slopes, "paper_slope_k2": 4.38 if ansatz == fp.BRICKWORK else None}


def fixed_topology(fp, torch, ansatz, n, depth, pairs, prec, seed, steps=3, chunk=None, local_dim=0):
    """Throughput of sample + contract + reduce for one fixed-topology ensemble; traces of the
    last step are returned for the precision comparison."""
    ens = fp.Ensemble(ansatz, n, depth, local_dim)
    chunk = chunk or pairs
    gates = fp.alloc_gates(ens, chunk, prec)
    trace = torch.empty(2 * pairs, dtype=torch.float64, device="cuda")
    ws = torch.empty(max(256, fp.fp_workspace_bytes(ens, chunk, prec)), dtype=torch.uint8, device="cuda")

    def step():
        for o in range(0, pairs, chunk):
            m = min(chunk, pairs - o)
            fp.fp_sample_gates(ens, m, seed, o, prec, gates)
            fp.fp_contract_trace_batch(ens, m, prec, gates, trace[2 * o: 2 * (o + m)], ws)
        return fp.fp_frame_potential(trace, pairs, 3)

    step()
    torch.cuda.synchronize()
    fp.fp_profile_begin()
    t0 = time.perf_counter()
    for _ in range(steps):
        f = step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = fp.fp_profile_end()
    kms = sum(prof[c]["ms"] for c in SWEEP_CLASSES)
    flops = sum(prof[c]["flops"] for c in SWEEP_CLASSES)
    progress(f"ensemble {ansatz}, n={n}, depth {depth}, precision {prec}: {pairs * steps / wall:.4g} pairs/s")
    return {"contractions_per_s": pairs * steps / wall, "F": f[0], "SE": f[1],
            "sweep_tflops": flops / (kms * 1e-3) / 1e12 if kms else 0.0,
            "kernel_ms_per_step": kms / steps}, trace


def precision_error(np, t32, t64, f32, f64):
    a = t32.cpu().numpy().reshape(-1, 2)
    b = t64.cpu().numpy().reshape(-1, 2)
    za, zb = a[:, 0] + 1j * a[:, 1], b[:, 0] + 1j * b[:, 1]
    rms = float(np.sqrt(np.mean(np.abs(zb) ** 2)))
    rel = np.abs(za - zb) / np.maximum(np.abs(zb), 1e-3 * rms)
    # the parity tests' complex64 reading: errors floored at the rms trace
    # (a float32 contraction's error is absolute on the scale of the traces)
    rel_rms = np.abs(za - zb) / np.maximum(np.abs(zb), rms)
    return {"max_floored_rel_trace_err": float(rel.max()), "median_rel_trace_err": float(np.median(rel)),
            "p99_rel_trace_err": float(np.quantile(rel, 0.99)),
            "max_rel_trace_err_floor_rms": float(rel_rms.max()),
            "rel_err_F_k": [abs(x - y) / abs(y) for x, y in zip(f32, f64)]}


def same_gate_precision(fp, torch, np, ens, gates_per_circuit, pairs, seed):
    """Contraction error of complex64 and BF16x3 against complex128 on the
    same gates: float32 gates are sampled once, and the complex128 run takes
    them widened to float64 (exactly), so only the contraction's rounding
    differs.  Haar ensembles only (the buffer holds 2 x gates_per_circuit
    4x4 complex gates per pair, then padding)."""
    e = fp.Ensemble(*ens)
    g32 = fp.sample(e, pairs, seed, 0, fp.C64)
    nb32, nb64 = fp.fp_gate_bytes_per_pair(e, fp.C64), fp.fp_gate_bytes_per_pair(e, fp.C128)
    nreal = 2 * gates_per_circuit * 32
    g64 = torch.zeros(pairs * nb64, dtype=torch.uint8, device="cuda")
    src = g32.view(pairs, nb32)[:, : 4 * nreal].contiguous().view(torch.float32)
    g64.view(pairs, nb64)[:, : 8 * nreal].view(torch.float64).copy_(src.to(torch.float64))
    out = {}
    for prec, buf in ((fp.C64, g32), (fp.C128, g64), (fp.BF16X3, g32)):
        out[prec] = fp.contract(e, buf, pairs, prec)
    f = {p: fp.frame_potential(out[p], 3)[0] for p in out}
    return {"pairs": pairs,
            "c64_vs_c128": precision_error(np, torch.view_as_real(out[fp.C64]), torch.view_as_real(out[fp.C128]),
                                           f[fp.C64], f[fp.C128]),
            "bf16x3_vs_c128": precision_error(np, torch.view_as_real(out[fp.BF16X3]),
                                              torch.view_as_real(out[fp.C128]), f[fp.BF16X3], f[fp.C128])}


def suite(fp, torch, np, synth, pairs):
    out = {}
    # brickwork n = 6, depths 1..6, 2000 pairs, complex128
    r = {}
    for d in range(1, 7):
        r[str(d)], _ = fixed_topology(fp, torch, fp.BRICKWORK, 6, d, 2000, fp.C128, synth.workload_seed(1, d))
    out["brickwork_n6_c128"] = r
    # brickwork n = 20, depths 2..10, complex64 and BF16x3 against complex128 on the same seeds
    r = {}
    keep = {}
    for d in range(2, 11):
        np_ = pairs if d <= 8 else max(1000, pairs // 20)
        seed = synth.workload_seed(2, d)
        steps = 3 if d <= 8 else 1
        r32, t32 = fixed_topology(fp, torch, fp.BRICKWORK, 20, d, np_, fp.C64, seed, steps=steps,
                                  chunk=min(np_, 20000))
        r64, t64 = fixed_topology(fp, torch, fp.BRICKWORK, 20, d, np_, fp.C128, seed, steps=1,
                                  chunk=min(np_, 20000))
        rb3, tb3 = fixed_topology(fp, torch, fp.BRICKWORK, 20, d, np_, fp.BF16X3, seed, steps=1,
                                  chunk=min(np_, 20000))
        r32["pairs"] = np_
        r32["c128_contractions_per_s"] = r64["contractions_per_s"]
        r32["bf16x3_contractions_per_s"] = rb3["contractions_per_s"]
        ngates = d // 2 * 9 + (d + 1) // 2 * 10  # 10 gates on odd layers, 9 on even ones (n = 20)
        r32["precision_same_gates"] = same_gate_precision(fp, torch, np, (fp.BRICKWORK, 20, d), ngates,
                                                          min(np_, 20000), seed)
        r[str(d)] = r32
        keep[d] = t32
    out["brickwork_n20"] = r
    out["brickwork_n20_layer_scaling"] = layer_scaling(fp, torch, keep, 20)
    progress(f"brickwork n=20 layers to epsilon = 0.1: "
             f"{ {k: round(v['median'], 2) for k, v in out['brickwork_n20_layer_scaling']['layers_to_epsilon'].items()} }")
    # HEA n = 30, layers 1..8, complex64
    r = {}
    for L in range(1, 9):
        r[str(L)], _ = fixed_topology(fp, torch, fp.HEA, 30, L, pairs, fp.C64, synth.workload_seed(3, L))
    out["hea_n30"] = r
    out["hea_n30_mixed_launch"] = hea_mixed(fp, torch, pairs)
    # the paper's hardware-efficient ansatz, CNOT walls against CZ walls,
    # n = 30, L = 1..7, complex64 (F^(k) falls toward k! faster with CNOT)
    for name, ans in (("pauli_cnot_n30", fp.PAULI_CNOT), ("pauli_cz_n30", fp.PAULI_CZ)):
        r = {}
        for L in range(1, 8):
            r[str(L)], _ = fixed_topology(fp, torch, ans, 30, L, pairs, fp.C64, synth.workload_seed(7 + ans, L))
        out[name] = r
    # qudit brickworks, n = 20, local dimension 3, 4, 5, every depth whose
    # register fits LDS, complex64 (F^(k) against k!, reached once q^n >= k)
    for q, dmax in ((3, 5), (4, 4), (5, 4)):
        r = {}
        for d in range(1, dmax + 1):
            r[str(d)], _ = fixed_topology(fp, torch, fp.BRICKWORK_QUDIT, 20, d, min(pairs, 20000), fp.C64,
                                          synth.workload_seed(10 + q, d), local_dim=q)
        out[f"qudit_q{q}_n20"] = r
    return out


def hea_mixed(fp, torch, pairs, steps=3):
    """The uneven-depth workload: HEA n = 30, L = 1..8, `pairs` pairs per L,
    in one fp_contract_trace_groups launch -- with the library's default
    launch choices, then with choices from fp_autotune -- against one
    fp_contract_trace_batch call per L on the same gates.  Contraction only
    (the gates are sampled beforehand); F^(1), F^(2) per L from the tuned
    launch."""
    import synth
    ens = [fp.Ensemble(fp.HEA, 30, L) for L in range(1, 9)]
    bufs = [fp.sample(e, pairs, synth.workload_seed(3, e.depth), 0, fp.C64) for e in ens]
    groups = [(i, fp.C64, 0, pairs) for i in range(len(ens))]
    tr = torch.empty(2 * pairs * len(ens), dtype=torch.float64, device="cuda")
    ws = torch.empty(max(256, fp.fp_workspace_bytes_groups(ens, groups)), dtype=torch.uint8, device="cuda")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return pairs * len(ens) * steps / (time.perf_counter() - t0)

    def mixed():
        fp.fp_contract_trace_groups(ens, groups, bufs, tr, ws)

    def per_l():
        for i, e in enumerate(ens):
            fp.fp_contract_trace_batch(e, pairs, fp.C64, bufs[i], tr[2 * i * pairs: 2 * (i + 1) * pairs])

    out = {"pairs_per_L": pairs, "default_mixed_launch_pairs_per_s": timed(mixed)}
    t0 = time.perf_counter()
    choices = {}
    for e in ens:
        c = fp.fp_autotune(e, fp.C64)
        choices[str(e.depth)] = [fp.AUTOTUNE_CLASSES[c // 3], fp.AUTOTUNE_TASK_FLOPS[c % 3]]
    out["autotune_s"] = time.perf_counter() - t0
    out["choices"] = choices
    out["tuned_mixed_launch_pairs_per_s"] = timed(mixed)
    out["per_L_calls_pairs_per_s"] = timed(per_l)
    mixed()
    out["F_per_L"] = {str(e.depth): fp.fp_frame_potential(tr[2 * i * pairs: 2 * (i + 1) * pairs], pairs, 2)[0]
                      for i, e in enumerate(ens)}
    progress(f"HEA n=30 L=1..8 mixed: default {out['default_mixed_launch_pairs_per_s']:.4g}, tuned "
             f"{out['tuned_mixed_launch_pairs_per_s']:.4g}, per-L calls {out['per_L_calls_pairs_per_s']:.4g} pairs/s")
    out["many_small_groups"] = hea_many_groups(fp, torch, steps)
    return out


def hea_many_groups(fp, torch, steps=3, n_groups=64, pairs=2000):
    """Uneven batches of many small groups: HEA n = 30, 64 groups of 2000
    pairs with L = 1..8 in turn (the tuning table of hea_mixed applies), in
    one fp_contract_trace_groups call against one fp_contract_trace_batch call
    per group on the same gates.  Contraction only."""
    import synth
    ens = [fp.Ensemble(fp.HEA, 30, 1 + g % 8) for g in range(n_groups)]
    bufs = [fp.sample(e, pairs, synth.workload_seed(30, g), 0, fp.C64) for g, e in enumerate(ens)]
    groups = [(g, fp.C64, 0, pairs) for g in range(n_groups)]
    tr = torch.empty(2 * pairs * n_groups, dtype=torch.float64, device="cuda")
    ws = torch.empty(max(256, fp.fp_workspace_bytes_groups(ens, groups)), dtype=torch.uint8, device="cuda")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return pairs * n_groups * steps / (time.perf_counter() - t0)

    def mixed():
        fp.fp_contract_trace_groups(ens, groups, bufs, tr, ws)

    def per_group():
        for g, e in enumerate(ens):
            fp.fp_contract_trace_batch(e, pairs, fp.C64, bufs[g], tr[2 * g * pairs: 2 * (g + 1) * pairs])

    out = {"groups": n_groups, "pairs_per_group": pairs, "mixed_launch_pairs_per_s": timed(mixed),
           "per_group_calls_pairs_per_s": timed(per_group)}
    progress(f"HEA n=30, {n_groups} groups of {pairs} pairs: one mixed call {out['mixed_launch_pairs_per_s']:.4g}, "
             f"per-group calls {out['per_group_calls_pairs_per_s']:.4g} pairs/s")
    return out


LR_MAX_BITS = 36  # widest slot of the HBM-slot sweep: 2^36 entries (64-bit entry indices beyond 2^31)


def planned_pairs(fp, np, n, s, seed_base, first, count):
    """Pairs first .. first + count - 1 of the local random workload at s
    steps, sampled by the product's sampler and planned by its host planner:
    the widest register of each pair and its complex multiply-adds."""
    ens = fp.Ensemble(fp.LOCAL_RANDOM, n, s)
    off = 2 * s * 32 * 4  # bonds follow the complex64 gates of U and V
    peaks, macs = [], []
    for lo in range(first, first + count, 1000):
        cnt = min(1000, first + count - lo)
        g = fp.sample(ens, cnt, seed_base | (s << 32), lo, fp.C64).view(cnt, -1)
        bonds = g[:, off: off + 8 * s].cpu().numpy()
        del g
        for p in range(cnt):
            b = np.frombuffer(bonds[p].tobytes(), dtype=np.int32).reshape(2, s)
            r = fp.fp_plan_local_random_host(n, b[0], b[1])
            peaks.append(r["peak_bits"])
            macs.append(r["macs"])
    return np.array(peaks), np.array(macs)


def feasibility(fp, np, n, depths, pairs, prec, seed_base, sample_arg):
    """Widest register of each pair in a sample per depth (the product's sampler
    and host planner on the sampled bonds), and the fraction of pairs beyond
    what one pair may take: 2^36 entries, and one slot of that width within
    the workspace the library asks for a batch of `pairs`.  The sample is a
    whole batch where the tail decides (a batch fits only if its widest pair
    does), smaller where most pairs are beyond anyway."""
    elem = 8 if prec == fp.C64 else 16
    out = {}
    for s in depths:
        sample = sample_arg or (pairs if s <= 400 else min(pairs, 2000))
        ens = fp.Ensemble(fp.LOCAL_RANDOM, n, s)
        pk, _ = planned_pairs(fp, np, n, s, seed_base, 0, sample)
        ws = fp.fp_workspace_bytes(ens, pairs, prec)
        budget = min(LR_MAX_BITS, int(math.floor(math.log2(ws / elem))))
        over = float(np.mean(pk > budget))
        top = int(pk.max())
        progress(f"widths at S={s}: {sample} pairs planned, widest 2^{int(pk.max())}")
        out[str(s)] = {
            "median_bits": int(np.quantile(pk, 0.5)), "p90_bits": int(np.quantile(pk, 0.9)),
            "p99_bits": int(np.quantile(pk, 0.99)), "max_bits": top, "sample_pairs": sample,
            "budget_bits": budget, "workspace_gib": ws / 2**30, "over_budget_frac": over,
            "status": "fits" if over == 0 else
                      f"infeasible: {int(round(over * sample))} of {sample} pairs ({over:.2%}) need more than "
                      f"2^{budget} entries per register (widest 2^{top} = {elem * 2.0 ** top / 2**30:.3g} GiB)",
        }
    return out


def _cpu_import(_):
    import oracle.mpo  # noqa: F401
    import oracle.sampler  # noqa: F401
    return 0


def _cpu_pair(args):
    depth, n, seed, pair = args
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass
    from oracle import mpo, sampler
    pr = sampler.sample_pairs(sampler.LOCAL_RANDOM, n, depth, seed, pair, 1, fp32=False)
    mpo.trace_pair(pr[0][0], pr[0][1])
    return 1


def cpu_baseline(n, depth, seed_base, seconds=8.0, runs=3):
    """The oracle (MPO-zip, complex128, with its own sampler) on a bounded
    sample: `runs` windows of `seconds` each over fresh pairs of the
    workload, handed out one at a time to one process per core the bench may
    use (at most 16 host threads per GPU).  Pairs still
    running at the end of a window are dropped with their processes (so the
    window's rate counts completed pairs only); the median window is
    reported."""
    import multiprocessing as mp
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    workers = max(1, min(16, avail))
    seed = seed_base | (depth << 32)
    rates, counts = [], []
    ctx = mp.get_context("spawn")
    for r in range(runs):
        pool = ctx.Pool(workers)
        try:
            pool.map(_cpu_import, range(workers), chunksize=1)  # start-up outside the window
            jobs = [(depth, n, seed, r * 100000 + i) for i in range(100000)]
            it = pool.imap_unordered(_cpu_pair, jobs, chunksize=1)
            t0 = time.perf_counter()
            done = 0
            while True:
                left = seconds - (time.perf_counter() - t0)
                if left <= 0:
                    break
                try:
                    done += it.next(timeout=left)
                except mp.TimeoutError:
                    break
            el = time.perf_counter() - t0
        finally:
            pool.terminate()
            pool.join()
        rates.append(done / el)
        counts.append(done)
    i = sorted(range(runs), key=lambda x: rates[x])[runs // 2]
    return {"value": rates[i], "unit": "contractions/s", "cores": workers, "nproc": os.cpu_count(),
            "cpus_available": avail, "kind": "oracle", "runs": [round(x, 4) for x in rates],
            "sample": f"median of {runs} windows of {seconds:g} s over fresh pairs of local random n={n} S={depth} "
                      f"(own Philox sampler + MPO-zip, complex128): {counts[i]} pairs completed, "
                      f"{workers} processes x 1 thread"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; sharding across GPUs is a design, not code",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2205_09900_amd as fp
    import synth

    torch.cuda.set_device(0)
    bench_streams(torch, max(1, args.in_flight))  # created together, before the library adds its side streams
    prec = fp.C64 if args.precision == "c64" else fp.C128
    seed_base = synth.workload_seed(4, 0)
    if args.with_copy:  # on a bench stream: the null stream takes no hardware queue of its own
        with torch.cuda.stream(bench_streams(torch, 1)[0]):
            a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
            b = torch.empty_like(a)
            b.copy_(a)
        torch.cuda.synchronize()

    # the step with one batch at a time, every launch timed with HIP events
    # (roofline and step breakdown); the same with batches in flight; and the
    # headline: batches in flight without events
    serial = run_workload(fp, torch, args.n, args.depth, args.pairs, prec, args.steps, 1, seed_base,
                          pipeline=False)
    if args.serial:
        head = timed = serial
    else:
        timed = run_workload(fp, torch, args.n, args.depth, args.pairs, prec, args.steps, args.warmup, seed_base,
                             in_flight=args.in_flight)
        head = run_workload(fp, torch, args.n, args.depth, args.pairs, prec, args.steps, args.warmup, seed_base,
                            in_flight=args.in_flight, profile=False)
    value = args.pairs * args.steps / head["wall_s"]
    prof = timed["prof"]
    # roofline of the sweep kernel with the largest event time (the sweeps
    # hold the method's arithmetic; planning, matrix preparation and sampling
    # are listed in step_kernels_ms), timed in the run with one batch at a
    # time: with batches in flight a kernel's events also span the other
    # batches' work on the GPU (that duration is reported beside it)
    sprof = serial["prof"]
    # the sweep class that does most of the step's algorithmic flops (the
    # longest launch can be a class with few pairs, e.g. the widest ones)
    dom = max(SWEEP_CLASSES, key=lambda c: sprof[c]["flops"])
    d = sprof[dom]
    peak = PEAK_FP32_TFLOPS if prec == fp.C64 else PEAK_FP64_TFLOPS
    achieved = (d["flops"] / d["launches"]) / (d["ms"] / d["launches"] * 1e-3) / 1e12 if d["launches"] else 0.0
    kname = LR_KERNELS[dom].format(r="float" if prec == fp.C64 else "double",
                                   big=1024 if prec == fp.C64 else 512)
    traffic = None
    from paper_2205_09900_amd import profile_summary
    summ = profile_summary.load_traffic(os.path.join(ROOT, "profiles", f"local_random_n{args.n}_S{args.depth}.md"))
    if summ and summ.get("workload") == f"local_random_n{args.n}_S{args.depth}_{args.precision}":
        traffic = summ["bytes_per_dispatch"].get(kname)
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": traffic, "kernel": kname, "kernel_class": dom,
                "kernel_ms_per_launch": d["ms"] / max(1, d["launches"]),
                "kernel_ms_per_launch_in_flight": prof[dom]["ms"] / max(1, prof[dom]["launches"]),
                "timed_in": "the run with one batch at a time (serial_ms_per_step)",
                "flops_per_launch": d["flops"] / max(1, d["launches"])}
    step_kernels = {c: {"ms_per_step": v["ms"] / args.steps, "launches_per_step": v["launches"] / args.steps,
                        "gflop_per_step": v["flops"] / args.steps / 1e9, "gb_per_step": v["bytes"] / args.steps / 1e9}
                    for c, v in prof.items() if v["launches"]}
    serial_kernels = {c: {"ms_per_launch": v["ms"] / v["launches"], "gflop_per_launch": v["flops"] / v["launches"] / 1e9}
                      for c, v in sprof.items() if v["launches"]}
    progress("one batch at a time, ms per launch: " + ", ".join(f"{c} {v['ms_per_launch']:.3f}"
                                                                  for c, v in serial_kernels.items()))

    per_depth = {}
    if args.per_depth:
        for s in [int(x) for x in args.per_depth.split(",") if x]:
            # step counts whose workspace takes most of the device (registers
            # beyond 2^31 entries) run one batch at a time, two batches
            deep = fp.fp_workspace_bytes(fp.Ensemble(fp.LOCAL_RANDOM, args.n, s), args.pairs, prec) > (64 << 30)
            fl = 1 if deep else args.in_flight
            depth_steps = 2 if deep else max(args.in_flight + 1, args.depth_steps)
            torch.cuda.empty_cache()
            r = run_workload(fp, torch, args.n, s, args.pairs, prec, depth_steps, 1 if not deep else 0, seed_base,
                             in_flight=fl, pipeline=not deep)
            r0 = run_workload(fp, torch, args.n, s, args.pairs, prec, depth_steps, 1 if not deep else 0, seed_base,
                              in_flight=fl, pipeline=not deep, profile=False)
            flops = sum(r["prof"][c]["flops"] for c in SWEEP_CLASSES)
            kms = sum(r["prof"][c]["ms"] for c in SWEEP_CLASSES)
            per_depth[str(s)] = {
                "contractions_per_s": args.pairs * depth_steps / r0["wall_s"],
                "contractions_per_s_with_events": args.pairs * depth_steps / r["wall_s"],
                "sweep_tflops": flops / (kms * 1e-3) / 1e12 if kms else 0.0,
                "F": r["F"], "SE": r["SE"], "batches": depth_steps, "batches_in_flight": fl,
                "kernel_ms_per_step": {k: v["ms"] / depth_steps for k, v in r["prof"].items()
                                       if v["launches"]},
            }

    # deeper step counts on small batches: the widest pairs set the time
    # there, so every batch is planned on the host first and one whose sweeps
    # would outlast the cap at a pessimistic rate is reported, not run
    if args.deep_depths and args.per_depth:
        for s in [int(x) for x in args.deep_depths.split(",") if x]:
            nb, npb = args.deep_batches, args.deep_pairs
            pk, macs = planned_pairs(fp, np, args.n, s, seed_base, 0, nb * npb)
            tflop = [8.0 * float(macs[i * npb:(i + 1) * npb].sum()) / 1e12 for i in range(nb)]
            est = [t / DEEP_PLAN_TFLOPS for t in tflop]
            entry = {"pairs_per_batch": npb, "batches": nb, "batches_in_flight": 1, "widest_bits": int(pk.max()),
                     "planned_tflop_per_batch": tflop, "planned_s_per_batch": est}
            if max(est) > args.deep_cap_s:
                entry["status"] = (f"not timed: a batch plans {max(tflop):.3g} TFLOP of sweeps, over "
                                   f"{args.deep_cap_s:g} s at {DEEP_PLAN_TFLOPS:g} TFLOP/s")
                progress(f"S={s}: {entry['status']}")
            else:
                torch.cuda.empty_cache()
                r = run_workload(fp, torch, args.n, s, npb, prec, nb, 0, seed_base, in_flight=1, pipeline=False,
                                 say_batches=True)
                flops = sum(r["prof"][c]["flops"] for c in SWEEP_CLASSES)
                kms = sum(r["prof"][c]["ms"] for c in SWEEP_CLASSES)
                entry.update({
                    "status": "measured (one run, with events)",
                    "contractions_per_s": npb * nb / r["wall_s"],
                    "sweep_tflops": flops / (kms * 1e-3) / 1e12 if kms else 0.0,
                    "F": r["F"], "SE": r["SE"], "F_per_batch": r["F_batches"],
                    "all_finite": bool(all(math.isfinite(x) for fb in r["F_batches"] for x in fb)),
                    "kernel_ms_per_step": {k: v["ms"] / nb for k, v in r["prof"].items() if v["launches"]},
                })
            per_depth[str(s)] = entry

    # register widths per depth, and which depths a batch fits: contractions/s
    # only where measured above, every other depth named with what it needs
    feas = {}
    if args.feasibility:
        feas = feasibility(fp, np, args.n, [int(x) for x in args.feasibility.split(",") if x], args.pairs, prec,
                           seed_base, args.feasibility_pairs)
        for k, v in feas.items():
            if k in per_depth and "contractions_per_s" in per_depth[k]:
                v["contractions_per_s"] = per_depth[k]["contractions_per_s"]
                v["status"] = "measured" if v["over_budget_frac"] == 0 else v["status"]
                per_depth[k].update({q: v[q] for q in ("median_bits", "p99_bits", "max_bits")})
            elif v["over_budget_frac"] == 0:
                v["status"] = "fits, not timed"

    suite_res = None
    if not args.no_suite:
        suite_res = suite(fp, torch, np, synth, args.suite_pairs)
        progress("other ensembles done")

    scaling_res = None
    if args.layer_scaling_n:
        scaling_res = layer_scaling_vs_n(fp, torch, np, synth, [int(x) for x in args.layer_scaling_n.split(",") if x],
                                         args.layer_scaling_pairs,
                                         fp.BRICKWORK if args.layer_scaling_ansatz == "brickwork" else fp.PAULI_CNOT)
        progress(f"layer scaling slopes in n: {scaling_res['slope_in_n']}")

    cv_res = None
    if not args.no_cv:
        from paper_2205_09900_amd import cv
        cv_res = cv.experiment(n=40, layers=6, k=2, hidden=256, n_train=65536, n_exact=10000,
                               n_surrogate=args.cv_surrogate, epochs=30)
        cv_res.pop("history", None)
        progress("control-variate experiment done")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.n, args.depth, seed_base, args.cpu_seconds)
        progress("CPU baseline done")

    config = {"workload": f"local_random_n{args.n}_S{args.depth}", "n_qubits": args.n,
              "steps_per_circuit": args.depth, "pairs_per_step": args.pairs, "k_max": 3,
              "precision": args.precision, "batches_in_flight": args.in_flight}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "contractions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["wall_s"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == fp.C64 else "f64",
        "data": "synthetic",
        "config": config,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    full = dict(out)
    full.update({
        "ms_per_step_with_events": timed["wall_s"] / args.steps * 1e3,
        "serial_ms_per_step": serial["wall_s"] / args.steps * 1e3,
        "serial_kernels": serial_kernels,
        "F_k": head["F"], "SE_k": head["SE"],
        "step_kernels_ms": step_kernels,
        "per_depth": per_depth,
        "feasibility": feas,
        "control_variate": cv_res,
        "ensembles": suite_res,
        "layer_scaling_vs_n": scaling_res,
    })
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(full, fh, indent=1)
        progress(f"full record written to {args.out}")
    # The stdout line stays small (the driver keeps only the tail of stdout):
    # the roofline without its bookkeeping, contractions/s per step count and
    # the control variate's two times; everything else is in --out.
    out["roofline"] = {k: roofline[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic", "kernel",
                                                "kernel_ms_per_launch")}
    out["F_k"] = [float(f"{x:.6g}") for x in head["F"]]
    out["per_S_contractions_per_s"] = {k: float(f"{v['contractions_per_s']:.4g}") for k, v in per_depth.items()
                                       if "contractions_per_s" in v}
    if cv_res:
        out["control_variate"] = {k: (float(f"{cv_res[k]:.4g}") if isinstance(cv_res[k], float) else cv_res[k])
                                  for k in ("workload", "time_to_1pct_plain_s", "time_to_1pct_cv_s", "rho_holdout",
                                            "used_control_variate") if k in cv_res}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
