"""Runs sample + contract + reduce on one ensemble (brickwork, local random,
HEA, Pauli-rotation HEA, qudit brickwork), for profiling single workloads
under rocprofv3 and for timing batches one after another.

    python -m paper_2205_09900_amd.run_ensemble --ansatz brickwork --n 20 --depth 2 \\
        --pairs 100000 --steps 5 [--precision c64] [--local-dim 3] [--with-copy]

Every step samples the pairs' gates (step i takes global pairs
[i P, (i+1) P)), contracts every pair and reduces F^(k), k = 1..3, on one
stream; --warmup steps (default 1) run untimed first, and every timed step
prints one progress line on stderr.  --with-copy also runs
one 256 MiB device copy, whose counter values calibrate FETCH_SIZE and
WRITE_SIZE (see profile_summary).  Prints one JSON line: pairs/s over the
timed steps, F^(k) and the sweep classes' event time and flops per step.
"""

import argparse
import json
import sys
import time

ANSATZ = {"brickwork": 0, "local_random": 1, "hea": 2, "pauli_cnot": 3, "pauli_cz": 4, "qudit": 5}
PRECISION = {"c128": 0, "c64": 1, "bf16x3": 2}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--ansatz", required=True, choices=sorted(ANSATZ))
    ap.add_argument("--n", type=int, required=True)
    ap.add_argument("--depth", type=int, required=True)
    ap.add_argument("--local-dim", type=int, default=0, help="q of a qudit brickwork")
    ap.add_argument("--pairs", type=int, default=100000)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="c64", choices=sorted(PRECISION))
    ap.add_argument("--seed", type=int, default=12345)
    ap.add_argument("--with-copy", action="store_true")
    args = ap.parse_args()

    import torch

    import paper_2205_09900_amd as fp

    ens = fp.Ensemble(ANSATZ[args.ansatz], args.n, args.depth, args.local_dim)
    prec = PRECISION[args.precision]
    if args.with_copy:
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    gates = fp.alloc_gates(ens, args.pairs, prec)
    trace = torch.empty(2 * args.pairs, dtype=torch.float64, device="cuda")
    ws = torch.empty(max(256, fp.fp_workspace_bytes(ens, args.pairs, prec)), dtype=torch.uint8, device="cuda")

    def step(i):
        fp.fp_sample_gates(ens, args.pairs, args.seed, i * args.pairs, prec, gates)
        fp.fp_contract_trace_batch(ens, args.pairs, prec, gates, trace, ws)
        return fp.fp_frame_potential(trace, args.pairs, 3)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    fp.fp_profile_begin()
    t0 = time.perf_counter()
    f = None
    for i in range(args.warmup, args.warmup + args.steps):
        f = step(i)
        print(f"[run_ensemble] step {i - args.warmup + 1}/{args.steps} done at "
              f"{time.perf_counter() - t0:.2f} s, F = {f[0]}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = fp.fp_profile_end()
    classes = {c: {"ms_per_step": v["ms"] / args.steps, "gflop_per_step": v["flops"] / args.steps / 1e9}
               for c, v in prof.items() if v["launches"]}
    print(json.dumps({"ensemble": repr(ens), "precision": args.precision, "pairs": args.pairs,
                      "steps": args.steps, "pairs_per_s": args.pairs * args.steps / wall,
                      "F": f[0], "SE": f[1], "classes": classes}))


if __name__ == "__main__":
    main()
