#!/usr/bin/env python
"""Benchmark of the dense Kohn-Sham path on one MI355X.

One step = one elsi_gpu_dm call on a fresh copy of (H, S) already resident in
HBM: Cholesky, reduction to standard form, full -> band -> tridiagonal,
divide and conquer, Fermi-Dirac chemical potential, back-transformations and
the density matrix (ELSI paper, Sec. 3.1 and 4.5).  Workload: the 3D
jittered-lattice Gaussian-basis system with N = 32768 basis functions,
n_occ = 8192, kT = 0.01 Ha, seed 0 (synthetic, standing in for the paper's
FHI-aims / DGDFT matrices).

The same line carries a `mixed` object: the same dm timed with FP32
matrix-core products in full -> band and Q1 followed by the FP64 refinement,
with its status and its deviation from the FP64 result (the metric's
comparison).

Prints one JSON line: throughput in algorithmic TFLOP/s,
F = 8/3 N^3 + 6 N^2 k_s (Cholesky N^3/3, reduction N^3, full -> band 4N^3/3,
two back-transformations 2 N^2 k each, back substitution N^2 k, density
matrix N^2 k_s, with k = k_s the eigenvectors that enter D), plus a
`roofline` object for the dominant kernel and a `cpu_baseline` object (the CPU
oracle timed on a bounded sample of the same workload).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GEVP+density-matrix wall time & TFLOP/s, N=32768: FP32+refine vs FP64 @1e-10 Ha"
WORKLOADS = {
    2: dict(n=32768, name="lattice3d_N32768_nocc8192_plain_fp64_dm"),
    1: dict(n=8192, name="lattice3d_N8192_nocc2048_plain_fp64_dm"),
}
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
GEMM_SRC = os.path.join(ROOT, "paper_1705_11191_amd", "csrc", "gemm.hip")
PROFILES = os.path.join(ROOT, "profiles")
# plain copy kernel used to calibrate the HBM byte counters: y = -x over
# COPY_ELEMS doubles reads and writes COPY_ELEMS * 8 bytes each
COPY_ELEMS = 1 << 28


def algorithmic_flops(n: int, ks: int) -> float:
    return (8.0 / 3.0) * n ** 3 + 6.0 * n * n * ks


FP32_PEAK_TFLOPS = 157.3   # MI355X dense FP32 matrix-core peak


def stage_roofline(stage_ms: dict, n: int, k: int, b: int, mixed: bool = False) -> dict:
    """Achieved rate of each stage against the peak of the unit it runs on.

    Algorithmic flops per stage (k = eigenvector columns the path carries for
    the density matrix, b = band width): Cholesky n^3/3, reduction n^3,
    full -> band 4n^3/3, bulge chasing 6 b n^2 (vector ALU, latency bound),
    Q2 and Q1 2 n^2 k each, back substitution n^2 k, density matrix n^2 k.
    `peak_of` names the unit whose peak `frac` is taken against; it says
    nothing about what bounds the stage (Q2 streams its columns from HBM).
    The matrix-core stages sum to 8/3 n^3 + 6 n^2 k, the benchmark's count.
    The divide-and-conquer merges and the refinement have no closed form
    here and carry their time only."""
    n3, n2k = float(n) ** 3, float(n) * n * k
    work = {"cholesky": (n3 / 3, "fp64_mfma"), "reduce": (n3, "fp64_mfma"), "band": (4 * n3 / 3, "fp64_mfma"),
            "bulge": (6.0 * b * n * n, "fp64_valu"), "back_q2": (2 * n2k, "fp64_mfma"),
            "back_q1": (2 * n2k, "fp64_mfma"), "backsub": (n2k, "fp64_mfma"), "density": (n2k, "fp64_mfma")}
    fp32_stages = ("band", "back_q1") if mixed else ()
    out = {}
    for st, ms in stage_ms.items():
        if st not in work or ms <= 0.0:
            out[st] = {"ms": ms}
            continue
        flops, unit = work[st]
        if st in fp32_stages:
            unit = "fp32_mfma"
        peak = FP32_PEAK_TFLOPS if unit == "fp32_mfma" else FP64_PEAK_TFLOPS   # FP64 vector peak = FP64 MFMA peak
        tf = flops / (ms * 1e-3) / 1e12
        out[st] = {"ms": ms, "flops": flops, "tflops": tf, "peak": peak, "frac": tf / peak, "peak_of": unit}
    return out


def _sha256(path: str) -> str:
    import hashlib

    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def _traffic_file(kernel: str, workload: str) -> str:
    tag = kernel.replace("<", "_").replace(">", "").replace(",", "_")
    return os.path.join(PROFILES, f"{tag}_{workload}_hbm_traffic.md")


def load_traffic(kernel: str, workload: str, launches: int):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None
    when there is none, the GEMM source changed since it was taken, or the solve
    now launches the kernel a different number of times (another mix of shapes)."""
    path = _traffic_file(kernel, workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic_json:"):
                rec = json.loads(line.split(":", 1)[1])
                if (rec.get("kernel") == kernel and rec.get("gemm_src_sha256") == _sha256(GEMM_SRC)
                        and rec.get("launches") == launches):
                    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    return None


def _pmc_rows(csv_path: str, counter: str):
    """(kernel name, value in KiB) per dispatch from a rocprofv3 counter_collection.csv."""
    import csv

    rows = []
    with open(csv_path, newline="") as fh:
        for r in csv.DictReader(fh):
            if r.get("Counter_Name") == counter:
                rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return rows


def summarize_pmc(fetch_csv: str, write_csv: str, kernel: str, workload: str, commands: list):
    """Write the per-launch HBM traffic summary of `kernel` (bytes), each counter
    scaled so that the calibration copy kernel reads/writes its known size."""
    known_kib = COPY_ELEMS * 8 / 1024.0
    out = {}
    for which, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        rows = _pmc_rows(path, counter)
        copies = [v for name, v in rows if "neg" in name.lower()]
        if not copies:
            raise SystemExit(f"{path}: no calibration copy dispatch found")
        # the calibration copy is the largest dispatch of the negation kernel
        factor = known_kib / max(copies)
        vals = [v for name, v in rows if _kernel_matches(name, kernel)]
        if not vals:
            raise SystemExit(f"{path}: no dispatch of {kernel}")
        out[which] = dict(factor=factor, launches=len(vals), kib_per_launch=sum(vals) / len(vals))
    rec = {
        "kernel": kernel,
        "workload": workload,
        "gemm_src_sha256": _sha256(GEMM_SRC),
        "fetch_bytes_per_launch": out["fetch"]["kib_per_launch"] * 1024 * out["fetch"]["factor"],
        "write_bytes_per_launch": out["write"]["kib_per_launch"] * 1024 * out["write"]["factor"],
        "fetch_factor": out["fetch"]["factor"],
        "write_factor": out["write"]["factor"],
        "launches": out["fetch"]["launches"],
    }
    path = _traffic_file(kernel, workload)
    with open(path, "w") as fh:
        fh.write(f"# HBM traffic of {kernel}, workload {workload}\n\n")
        fh.write("Counters: FETCH_SIZE and WRITE_SIZE (KiB per dispatch), one rocprofv3 pass each.\n")
        fh.write(f"Calibration: a plain copy kernel (y = -x over {COPY_ELEMS} doubles, "
                 f"{COPY_ELEMS * 8} bytes each way) in the same run; factor = known size / counter.\n\n")
        fh.write("Commands:\n\n")
        for c in commands:
            fh.write(f"    {c}\n")
        fh.write("\n")
        fh.write(f"| counter | launches | KiB/launch (raw) | factor | bytes/launch |\n|---|---|---|---|---|\n")
        fh.write(f"| FETCH_SIZE | {out['fetch']['launches']} | {out['fetch']['kib_per_launch']:.1f} | "
                 f"{out['fetch']['factor']:.4f} | {rec['fetch_bytes_per_launch']:.4g} |\n")
        fh.write(f"| WRITE_SIZE | {out['write']['launches']} | {out['write']['kib_per_launch']:.1f} | "
                 f"{out['write']['factor']:.4f} | {rec['write_bytes_per_launch']:.4g} |\n\n")
        fh.write("traffic_json: " + json.dumps(rec) + "\n")
    print(path)


def _kernel_matches(full_name: str, short: str) -> bool:
    """rocprofv3 prints e.g. 'void eg::(anonymous namespace)::dgemm_kernel<128, 128, 0, true, false, false>(...)'."""
    return full_name.replace(" ", "").find(short.replace(" ", "") + "(") >= 0


def cpu_model() -> str:
    """The host CPU's model name (first 'model name' line of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_sample: int):
    """The CPU oracle (plain C, OpenMP) on a bounded sample of the same workload."""
    import numpy as np

    import oracle
    from synth import generator as G

    sp = G.make_lattice_system(n_sample, seed=0)
    t0 = time.perf_counter()
    r = oracle.dm(sp.H, sp.S, sp.n_occ, sp.kT)
    dt = time.perf_counter() - t0
    ks = int(np.sum(r["occ"] > 1e-20))
    cores = int(os.environ.get("OMP_NUM_THREADS", 0)) or os.cpu_count()
    return {
        "value": algorithmic_flops(n_sample, ks) / dt / 1e12,
        "unit": "TFLOP/s",
        "cores": cores,
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": (f"one oracle dm solve of the same 3D-lattice generator at N={n_sample} "
                   f"(n_occ={n_sample // 4}, k_s={ks}), {dt:.1f} s; rate = algorithmic flops / time"),
    }


def batch_bench(args):
    """256 independent lattice problems, sizes log-uniform in [256, 4096] rounded
    to multiples of 15, problem i from seed i, n_occ = n // 4: one batched dm
    call vs a loop of single-problem dm calls (band width 64) on the same
    inputs.  With --tune, the tuner first picks the batched calls' band width
    per size bucket on samples of this batch (outside the timed steps)."""
    import torch

    from paper_1705_11191_amd import binding as B
    from synth import generator as G

    dev = torch.device("cuda:0")
    sizes = [int(x) for x in G.batch_sizes(args.batch_count, seed=0)]
    t_gen = time.perf_counter()
    H0, S0, nocc = [], [], []
    for i, n in enumerate(sizes):
        sp = G.make_lattice_system(n, seed=i, device=dev)
        H0.append(sp.H)
        S0.append(sp.S)
        nocc.append(sp.n_occ)
    torch.cuda.synchronize()
    print(f"[bench] {len(sizes)} batch inputs built in {time.perf_counter() - t_gen:.1f} s "
          f"(sum n = {sum(sizes)})", file=sys.stderr, flush=True)
    H = [torch.empty_like(x) for x in H0]
    S = [torch.empty_like(x) for x in S0]
    h = B.Handle(8, 8, 2)
    h.set_batch_workers(args.batch_workers)
    tuned = None
    if args.tune:
        # the band width per size bucket, timed on samples of this batch (not part of the timed steps)
        from paper_1705_11191_amd import tune

        tuned = tune.tune_batch_band_widths(h, H0, S0, nocc, workers=args.batch_workers,
                                            cache_path=args.tune_cache,
                                            log=lambda m: print(m, file=sys.stderr, flush=True))
        print(f"[bench] band widths per bucket: {tuned['n_max']} -> {tuned['b']} "
              f"({tuned['tune_ms']:.0f} ms of tuning)", file=sys.stderr, flush=True)

    def batched():
        for a, b in zip(H, H0):
            a.copy_(b)
        for a, b in zip(S, S0):
            a.copy_(b)
        return h.dm_batched(H, S, nocc)

    for w in range(args.warmup):
        batched()
        print(f"[bench] batched warmup {w} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        Ds, evals, energy, mu, status, rc = batched()
        print(f"[bench] batched step {k} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ms_batched = (time.perf_counter() - t0) * 1e3 / args.steps
    # the same problems one call at a time (the single-problem path): one
    # handle per size, created and warmed (workspace allocated, first launches
    # done) by an untimed pass, then one timed pass
    hs = {}
    for i, n in enumerate(sizes):
        if n not in hs:
            hs[n] = B.Handle(n, n, nocc[i])
    D_seq = [B.fortran_empty(n, n, device=dev) for n in sizes]

    def sequential():
        for i, n in enumerate(sizes):
            H[i].copy_(H0[i])
            S[i].copy_(S0[i])
            hs[n].dm(H[i], S[i], D_out=D_seq[i])

    sequential()
    torch.cuda.synchronize()
    print("[bench] sequential warm-up pass done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    sequential()
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - t0) * 1e3
    print(f"[bench] sequential loop done: {ms_seq:.1f} ms", file=sys.stderr, flush=True)
    maxdiff = max(float((a - b).abs().max().item()) for a, b in zip(Ds, D_seq))
    # k_s per problem: states with a Fermi-Dirac occupation above 1e-20 at the returned mu
    kT = 0.01
    ks = [int(((ev - m) / kT < 46.0517).sum().item()) for ev, m in zip(evals, mu)]
    F = sum(algorithmic_flops(n, k) for n, k in zip(sizes, ks))
    for hh in hs.values():
        hh.close()
    h.close()
    out = {
        "metric": "batched GEVP+density-matrix wall time & TFLOP/s, 256 problems n in [255, 4095]",
        "value": F / (ms_batched / 1e3) / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_batched,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"lattice3d_batch{len(sizes)}_loguniform256_4096_plain_fp64_dm",
                   "problems": len(sizes), "sum_n": sum(sizes), "workers": args.batch_workers,
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))},
        "band_table": ({"n_max": tuned["n_max"], "b": tuned["b"], "tune_ms": tuned["tune_ms"],
                        "cached": tuned["cached"]} if tuned else None),
        "sequential_single_calls_ms": ms_seq,
        "sequential_note": "one warmed handle per size, created outside the timed pass",
        "speedup_vs_sequential": ms_seq / ms_batched,
        "checks": {"status_all_zero": all(x == 0 for x in status),
                   "max_abs_D_batched_minus_single": maxdiff},
    }
    print(json.dumps(out), flush=True)


def complex_bench(args):
    """Complex Hermitian k-point problems: the periodic 8 x 8 x 12 cell of
    s-Gaussians (768 atoms x 15 = 11,520 basis functions), Bloch sums over the
    27 nearest images, the first args.kpoints points of the 4 x 2 x 2
    Monkhorst-Pack grid without Gamma, n_occ = N / 4 per cell, one
    complex-handle dm call per k-point per step.  Flops are counted as for a
    complex solver, 4 F(N, k_s) per k-point; the library solves the real
    2N x 2N image, which takes twice that."""
    import torch

    from paper_1705_11191_amd import binding as B
    from synth import generator as G

    dev = torch.device("cuda:0")
    cell = tuple(int(x) for x in args.cell.split(","))
    kpts = G.MP_KPOINTS_4x2x2[: args.kpoints]
    t_gen = time.perf_counter()
    H0, S0 = [], []
    for q, k in enumerate(kpts):
        sp = G.make_kpoint_system_torch(cell, k, seed=0, device=dev)
        H0.append(sp.H)
        S0.append(sp.S)
        nocc = sp.n_occ
        kT = sp.kT
    torch.cuda.synchronize()
    n = int(H0[0].shape[0])
    print(f"[bench] {len(kpts)} k-point inputs (N = {n} complex) built in {time.perf_counter() - t_gen:.1f} s",
          file=sys.stderr, flush=True)
    mixed = args.precision == "mixed"
    h = B.Handle(n, n, nocc, dtype=B.COMPLEX128)
    h.set_band_width(args.band)
    if mixed:
        h.set_precision(B.PREC_MIXED, args.refine_tol, args.max_refine)
    ok = (0, 3) if mixed else (0,)
    if args.shared_mu:
        # all k-points in one batched call with weights 1/nk: one mu for the cell
        h.set_batch_workers(max(1, min(args.batch_workers, 2)))
        Hb = [B.fortran_empty(n, n, device=dev, dtype=torch.complex128) for _ in kpts]
        Sb = [B.fortran_empty(n, n, device=dev, dtype=torch.complex128) for _ in kpts]
        wk = [1.0 / len(kpts)] * len(kpts)

        def step():
            for q in range(len(kpts)):
                Hb[q].copy_(H0[q])
                Sb[q].copy_(S0[q])
            Ds, evs, energies, mus, status, rc = h.dm_batched(Hb, Sb, [nocc] * len(kpts), kweight=wk, ok=ok)
            kts = [int(((ev - mus[0]) / kT < 46.0517).sum().item()) for ev in evs]
            return [(ev, e, m, st, kk) for ev, e, m, st, kk in zip(evs, energies, mus, status, kts)], Ds
    else:
        H = B.fortran_empty(n, n, device=dev, dtype=torch.complex128)
        S = B.fortran_empty(n, n, device=dev, dtype=torch.complex128)
        D = B.fortran_empty(n, n, device=dev, dtype=torch.complex128)

        def step():
            outs = []
            for q in range(len(kpts)):
                H.copy_(H0[q])
                S.copy_(S0[q])
                Dq, ev, f, energy, mu, st = h.dm(H, S, D_out=D, ok=ok)
                outs.append((ev, energy, mu, st, h.info()["k_s"]))
            return outs, [D]

    for w in range(args.warmup):
        step()
        print(f"[bench] complex warmup {w} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        outs, Dl = step()
        print(f"[bench] complex step {k} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    F = sum(4.0 * algorithmic_flops(n, o[4]) for o in outs)
    # checks on the last k-point: D Hermitian, tr(D S) = n_occ (times its weight with a shared mu)
    D = Dl[-1]
    herm = float((D - D.conj().t()).abs().max().item())
    if args.shared_mu:   # the weighted occupations put the cell's electrons into sum_k tr(D_k S_k)
        trDS = sum(complex((Dq * Sq.t()).sum().item()) for Dq, Sq in zip(Dl, S0))
    else:
        trDS = complex((D * S0[-1].t()).sum().item())
    h.close()
    out = {
        "metric": "complex Hermitian GEVP+density-matrix wall time & TFLOP/s (complex flop count)",
        "value": F / (ms / 1e3) / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": f"kpoint3d_cell{cell[0]}x{cell[1]}x{cell[2]}_N{n}_k{len(kpts)}_complex_dm"
                               + ("_shared_mu" if args.shared_mu else "") + ("_mixed" if mixed else ""),
                   "n_basis": n, "kpoints": len(kpts), "n_occ": int(nocc), "kT_Ha": kT,
                   "band_width": args.band, "path": "real 2N image",
                   "mu": "shared over k-points (weights 1/nk)" if args.shared_mu else "per k-point",
                   "precision": "fp32 products + fp64 refinement" if mixed else "fp64"},
        "ms_per_kpoint": ms / len(kpts),
        "k_s": [o[4] for o in outs],
        "mu_Ha": [o[2] for o in outs],
        "checks": {"status_all_zero": all(o[3] == 0 for o in outs), "D_hermitian_max_abs": herm,
                   "trace_DS_minus_Ne_last": trDS.real - nocc, "trace_DS_imag_last": trDS.imag},
    }
    print(json.dumps(out), flush=True)


def counters_q2(args):
    """The counter passes' Q2 program: a calibration copy (--calibrate-copy),
    then X <- Q X for a random symmetric A of order n and n/2 columns."""
    import torch

    from paper_1705_11191_amd import binding as B

    n = args.counters_n
    if args.calibrate_copy:
        x = torch.ones(COPY_ELEMS, device="cuda", dtype=torch.float64)
        y = torch.empty_like(x)
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        del x, y
    g = torch.Generator(device="cuda").manual_seed(5)
    A = torch.randn(n, n, device="cuda", dtype=torch.float64, generator=g)
    A = A + A.T
    X = B.fortran_empty(n, n // 2)
    X.copy_(torch.randn(n, n // 2, device="cuda", dtype=torch.float64, generator=g))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.backtransform(A, args.band, X, trans=False)
    torch.cuda.synchronize()
    print(json.dumps({"counters_only": True, "stage": "q2", "n": n, "ncol": n // 2,
                      "wall_s": time.perf_counter() - t0}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2, choices=sorted(WORKLOADS))
    ap.add_argument("--band", type=int, default=64)
    ap.add_argument("--cpu-sample-n", type=int, default=3072)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain copy kernel of known size first (HBM counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM traffic summary of --kernel from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--kernel", default="dgemm_kernel<128,128,0,true,false,false>")
    ap.add_argument("--counters-only", action="store_true",
                    help="one untimed FP64 step of the single workload and nothing else (no HIP events, no "
                         "launch probe, no CPU baseline): the program the hardware-counter passes run")
    ap.add_argument("--counters-stage", choices=["dm", "q2"], default="dm",
                    help="with --counters-only: dm (the whole solve of the workload) or q2 (one application "
                         "of Q = Q1 Q2 to n/2 columns, n = --counters-n, random symmetric input)")
    ap.add_argument("--counters-n", type=int, default=16384)
    ap.add_argument("--pmc-command", action="append", default=[])
    ap.add_argument("--workload", choices=["single", "batch", "complex"], default="single",
                    help="single: the N=32768 dm solve; batch: 256 uneven problems in one batched call")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--kpoints", type=int, default=4, help="complex workload: k-points per step (1..16)")
    ap.add_argument("--shared-mu", action="store_true",
                    help="complex workload: one batched call over the k-points with one chemical potential")
    ap.add_argument("--cell", default="8,8,12", help="complex workload: cell sites along x,y,z")
    ap.add_argument("--batch-workers", type=int, default=16)
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="batch workload: hardware queues of the HIP runtime (GPU_MAX_HW_QUEUES, read when "
                         "the runtime starts; worker streams beyond it share queues); 0 keeps the environment's")
    ap.add_argument("--tune", action="store_true",
                    help="batch workload: tune the band width per size bucket before the timed steps")
    ap.add_argument("--tune-cache", default=None,
                    help="batch workload: JSON cache of tuned band-width tables (default: $ELSI_GPU_TUNE_CACHE)")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="single workload: fp64 times plain FP64 (headline) and, unless --no-mixed, the mixed "
                         "path beside it; mixed times only FP32 matrix-core products in full -> band and Q1 "
                         "followed by FP64 refinement")
    ap.add_argument("--refine-tol", type=float, default=1e-10)
    ap.add_argument("--max-refine", type=int, default=6)
    ap.add_argument("--no-mixed", action="store_true",
                    help="single workload: skip the FP32+refine run that the default line reports beside FP64")
    ap.add_argument("--mixed-steps", type=int, default=1,
                    help="single workload: timed steps of the FP32+refine run (after one warm-up)")
    args = ap.parse_args()
    if args.workload == "batch" and args.hw_queues > 0:
        # read by the HIP runtime when it starts, i.e. before torch touches the GPU
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(args.hw_queues, 32))
    if args.workload == "complex":
        if args.gpus != 1:
            print("bench.py measures one GPU only", file=sys.stderr)
            sys.exit(2)
        complex_bench(args)
        return
    if args.workload == "batch":
        if args.gpus != 1:
            print("bench.py measures one GPU only", file=sys.stderr)
            sys.exit(2)
        batch_bench(args)
        return
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.kernel,
                      WORKLOADS[args.config]["name"], args.pmc_command)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the path has no multi-GPU mode); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1705_11191_amd import binding as B
    from synth import generator as G

    if args.counters_only and args.counters_stage == "q2":
        counters_q2(args)
        return
    wl = WORKLOADS[args.config]
    n = wl["n"]
    dev = torch.device("cuda:0")
    t_gen = time.perf_counter()
    spec = G.make_lattice_system(n, seed=0, device=dev)
    H0, S0 = spec.H, spec.S
    torch.cuda.synchronize()
    print(f"[bench] inputs N={n} built in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    n_occ = spec.n_occ
    H = torch.empty_like(H0)
    S = torch.empty_like(S0)
    D = torch.empty_like(H0)
    ev = torch.empty(n, device=dev, dtype=torch.float64)
    f = torch.empty(n, device=dev, dtype=torch.float64)

    if args.calibrate_copy:
        x = torch.ones(COPY_ELEMS, device=dev, dtype=torch.float64)
        y = torch.empty_like(x)
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        del x, y

    def run_path(mixed: bool, steps: int, warmup: int, probe: bool):
        """warmup + timed steps of one path on a fresh handle; then, when probe,
        one more step with HIP events around every GEMM launch (a separate,
        untimed pass, so the headline carries no probe overhead)."""
        h = B.Handle(n, n, n_occ)
        h.set_band_width(args.band)
        if mixed:
            h.set_precision(B.PREC_MIXED, args.refine_tol, args.max_refine)
        ws = torch.empty(h.workspace_size() // 8 + 1, device=dev, dtype=torch.float64)
        h.set_workspace(ws)
        status = [0]
        tag = "mixed" if mixed else "fp64"

        def step():
            H.copy_(H0)
            S.copy_(S0)
            r = h.dm(H, S, occ=f, D_out=D, eval_out=ev, ok=(0, 3) if mixed else (0,))
            status[0] = r[5]
            return r

        for w in range(warmup):
            step()
            print(f"[bench] {tag} warmup {w} done: {h.info()['total_ms']:.1f} ms", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stage_ms = None
        for k in range(steps):
            step()
            inf = h.info()
            print(f"[bench] {tag} step {k}: {inf['total_ms']:.1f} ms", file=sys.stderr, flush=True)
            if stage_ms is None:
                stage_ms = {st: 0.0 for st in inf["stage_ms"]}
            for st, v in inf["stage_ms"].items():
                stage_ms[st] += v / steps
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        info = h.info()
        probe_info = None
        if probe:
            h.set_launch_timing(True)   # HIP events around each GEMM launch, on the library's stream
            step()
            probe_info = h.info()
            h.set_launch_timing(False)
            print(f"[bench] {tag} probe step: {probe_info['total_ms']:.1f} ms", file=sys.stderr, flush=True)
        h.close()
        del ws
        return ms, stage_ms, info, probe_info, status[0]

    if args.counters_only:
        # the calibration copy (--calibrate-copy) ran above; one plain step follows
        t0 = time.perf_counter()
        run_path(False, 1, 0, probe=False)
        print(json.dumps({"counters_only": True, "workload": wl["name"],
                          "wall_s": time.perf_counter() - t0}), flush=True)
        return
    mixed_only = args.precision == "mixed"
    out = None
    ref64 = None
    if not mixed_only:
        ms, stage_ms, info, pinfo, _ = run_path(False, args.steps, args.warmup, probe=True)
        ks = info["k_s"]
        F = algorithmic_flops(n, ks)
        value = F / (ms / 1e3) / 1e12
        kname = pinfo["probe_kernel"]
        launches = max(pinfo["probe_launches"], 1)
        achieved = pinfo["probe_flops"] / (pinfo["probe_ms"] * 1e-3) / 1e12 if pinfo["probe_ms"] > 0 else 0.0
        roofline = {
            "bound": "mfma",
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": load_traffic(kname, wl["name"], pinfo["probe_launches"]),
            "kernel": kname,
            "launches_per_step": pinfo["probe_launches"],
            "avg_launch_ms": pinfo["probe_ms"] / launches,
            "flops_per_launch": pinfo["probe_flops"] / launches,
            "measured": "HIP events around every launch of the kernel on the library's stream, over one step "
                        "run after the timed steps",
        }
        # quick invariants on the last step: tr(D S) = N_e, ascending eigenvalues
        trace_ds = float((D * S0).sum().item())
        ascending = bool(torch.all(ev[1:] >= ev[:-1]).item())
        out = {
            "metric": METRIC,
            "value": value,
            "unit": "TFLOP/s",
            "n_gpus": 1,
            "steps": args.steps,
            "warmup": args.warmup,
            "ms_per_step": ms,
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": wl["name"], "n_basis": n, "n_occ": int(n_occ), "kT_Ha": spec.kT,
                       "kappa_S": spec.meta["kappa"], "band_width": info["band_width"], "k_s": ks,
                       "path": "plain_fp64"},
            "roofline": roofline,
            "algorithmic_flops": F,
            "stage_ms": stage_ms,
            "stage_roofline": stage_roofline(stage_ms, n, ks, info["band_width"], False),
            "checks": {"trace_DS_minus_Ne": trace_ds - n_occ, "eigenvalues_ascending": ascending,
                       "mu_Ha": info["mu"]},
        }
    if not args.no_mixed:
        if out is not None:
            ref64 = (D.clone(), ev.clone(), out["config"]["k_s"])
        else:
            # untimed FP64 solve of the same input: the accuracy yardstick of the mixed path
            _, _, info64, _, _ = run_path(False, 1, 0, probe=False)
            ref64 = (D.clone(), ev.clone(), info64["k_s"])
        torch.cuda.empty_cache()
        msteps = args.steps if mixed_only else args.mixed_steps
        ms_m, stage_m, info_m, _, st_m = run_path(True, msteps, args.warmup if mixed_only else 1, probe=False)
        D64, ev64, ks64 = ref64
        ks_m = info_m["k_s"]
        kk = min(ks_m, ks64)
        F_m = algorithmic_flops(n, ks_m)
        mixed = {
            "path": "fp32_products_fp64_refine",
            "ms_per_step": ms_m,
            "steps": msteps,
            "tflops_algorithmic": F_m / (ms_m / 1e3) / 1e12,
            "status": st_m,
            "refine_sweeps": info_m["refine_sweeps"],
            "refine_states": info_m["refine_states"],
            "refine_step": info_m["refine_step"],
            "refine_tol": args.refine_tol,
            "residual_Ha": info_m["refine_resid"],
            "k_s": ks_m,
            "max_abs_dD_vs_fp64": float((D - D64).abs().max().item()),
            "max_abs_deig_vs_fp64_Ha": float((ev[:kk] - ev64[:kk]).abs().max().item()),
            "stage_ms": stage_m,
            "stage_roofline": stage_roofline(stage_m, n, ks_m, info_m["band_width"], True),
        }
        if out is not None:
            mixed["speedup_vs_fp64"] = out["ms_per_step"] / ms_m
            out["mixed"] = mixed
        else:
            out = {
                "metric": METRIC,
                "value": F_m / (ms_m / 1e3) / 1e12,
                "unit": "TFLOP/s",
                "n_gpus": 1,
                "steps": msteps,
                "warmup": args.warmup,
                "ms_per_step": ms_m,
                "higher_is_better": True,
                "scaling": "weak",
                "vs_baseline": None,
                "dtype": "f32+f64",
                "data": "synthetic",
                "config": {"workload": wl["name"].replace("plain_fp64", "mixed"), "n_basis": n,
                           "n_occ": int(n_occ), "kT_Ha": spec.kT, "kappa_S": spec.meta["kappa"],
                           "band_width": info_m["band_width"], "k_s": ks_m, "path": "fp32_products_fp64_refine"},
                "mixed": mixed,
            }
        del ref64, D64, ev64
    del H, S, D, H0, S0
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_n)
        out["cpu_baseline_note"] = "the CPU baseline is the FP64 oracle, for both precisions"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
