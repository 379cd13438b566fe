"""Benchmark of the even-odd Schur Dirac apply (and the solves built on it) on one MI355X.

Workload: 32^3 x 64 lattice, synthetic SU(3) x U(1) fields (eps = 0.5, theta in (-0.3, 0.3)),
kappa = 0.1245, c_sw = 1.6, c_sw^QED = 1.0, qhat = -1, antiperiodic time.  One step is one
application of the even-odd Schur operator D-hat in FP64 on the NATIVE layout, inputs resident
in HBM.  Prints one JSON line on stdout; diagnostics go to stderr.

Algorithmic bytes (each field read once, output written once, links as 12 reals + 1 angle):
  Schur D-hat   472 reals per even site  (3776 B in FP64, 1888 B in FP32)
  hop + A_ee chi (second Schur kernel)  248 reals per site (1984 B FP64)
  hop + A_oo^-1  (first Schur kernel)   224 reals per site (1792 B FP64)
Also reported: FP32/FP16/BF16 and C* Schur applies, 12 right-hand sides in one call, the Schur
apply at 48^3 x 12 (one GPU's share of 48^3 x 96 cut along t over 8 GPUs), and the solves.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DIMS = (64, 32, 32, 32)  # (L0 = time, L1, L2, L3)
KAPPA, CSW, CSW_QED, QHAT, EPS, SEED = 0.1245, 1.6, 1.0, -1, 0.5, 201
SCHUR_REALS, CLOV_HOP_REALS, INV_HOP_REALS = 472, 248, 224
FLOP_SCHUR, FLOP_HOP, FLOP_CLOVER = 3672, 1320, 504


# launch shapes of the hop kernel, in the library's order (index = the tuner's choice)
HOP_SHAPES = ["k_hop_p bs256 1/CU 2 neighbours/iteration streaming hints (persistent)",
              "k_hop_p bs256 1/CU streaming hints (persistent)", "k_hop_p bs256 2/CU streaming hints (persistent)",
              "k_hop_p bs256 1/CU (persistent)", "k_hop_p bs256 1/CU 2 neighbours/iteration (persistent)",
              "k_hop bs256 xcd-order", "k_hop bs256", "k_hop bs128 xcd-order", "k_hop bs64 xcd-order",
              "k_hop_t tt4 (time-tiled LDS)", "k_hop_t tt8 (time-tiled LDS)", "k_hop_p bs512 1/CU (persistent)",
              "k_hop_p bs256 2/CU (persistent)", "k_hop_p bs256 1/CU xcd-regions (persistent)",
              "k_hop_tp tt4 1/CU (persistent time-tiled)", "k_hop_tp tt8 1/CU (persistent time-tiled)",
              "k_hop_ps bs256 1/CU (XCD slab sweep)", "k_hop_ps bs256 2/CU (XCD slab sweep)",
              "k_hop_ps bs128 2/CU (XCD slab sweep)", "k_hop_p bs256 2/CU 2 neighbours/iteration (persistent)",
              "k_hop_mr 2 RHS/work-item 1/CU streaming hints", "k_hop_mr 4 RHS/work-item 1/CU streaming hints",
              "k_hop_mr 2 RHS/work-item 2/CU streaming hints",
              "k_hop_rb 4 waves (right-hand sides blocked, link work and clover in LDS)",
              "k_hop_rb 8 waves (right-hand sides blocked, link work and clover in LDS)",
              "k_hop_rb 4 waves, next-direction prefetch", "k_hop_rb 8 waves, next-direction prefetch",
              "k_hop_rb 12 waves, next-direction prefetch",
              "k_hop_p bs256 1/CU 4 neighbours/iteration streaming hints (persistent)",
              "k_hop_p bs256 2/CU 4 neighbours/iteration streaming hints (persistent)",
              "k_hop_px bs256 1/CU 2 neighbours/iteration streaming hints (x1-split sweep)",
              "k_hop_px bs256 2/CU 2 neighbours/iteration streaming hints (x1-split sweep)",
              "k_hop_px bs128 2/CU 2 neighbours/iteration streaming hints (x1-split sweep)",
              "k_hop_px bs256 1/CU 4 neighbours/iteration streaming hints (x1-split sweep)",
              "k_hop_ps bs256 1/CU 2 neighbours/iteration streaming hints (XCD slab sweep)",
              "k_hop_ps bs128 2/CU 2 neighbours/iteration streaming hints (XCD slab sweep)",
              "k_hop_px bs256 2/CU 4 neighbours/iteration streaming hints (x1-split sweep)",
              "k_hop_px bs256 4/CU 2 neighbours/iteration streaming hints (x1-split sweep)",
              "k_hop_rb 4 waves, next-direction prefetch, x1-split block order",
              "k_hop_rb 8 waves, next-direction prefetch, x1-split block order",
              "k_hop_px bs256 3/CU 4 neighbours/iteration streaming hints (x1-split sweep)",
              "k_hop_rbc 12 waves x 1 RHS, column walk, x1-split", "k_hop_rbc 8 waves x 2 RHS, column walk, x1-split",
              "k_hop_rbc 4 waves x 3 RHS, 2/CU, column walk, x1-split", "k_hop_rbc 6 waves x 2 RHS, column walk, x1-split",
              "k_hop_rbc 12 waves x 1 RHS, column walk",
              "k_hop_rbc 12 waves x 1 RHS, column walk, x1-split, double-buffered LDS",
              "k_hop_rbc 8 waves x 2 RHS, column walk, x1-split, double-buffered LDS"]

# The FP64 hop + A chi kernel of each launch shape, as rocprofv3 names it, and its grid in
# work-items on 32^3 x 64 (V/2 = 1,048,576 output sites, 256 compute units): the key of its row in
# the committed counter summary, from which the roofline's HBM traffic is read.
HOP_CLOV_KERNEL_32C64 = {
    0: ("k_hop_p<double, 0, 2, 256, 0, 2, true>", 65536), 1: ("k_hop_p<double, 0, 2, 256, 0, 1, true>", 65536),
    2: ("k_hop_p<double, 0, 2, 256, 0, 1, true>", 131072), 3: ("k_hop_p<double, 0, 2, 256, 0, 1, false>", 65536),
    4: ("k_hop_p<double, 0, 2, 256, 0, 2, false>", 65536), 11: ("k_hop_p<double, 0, 2, 512, 0, 1, false>", 131072),
    12: ("k_hop_p<double, 0, 2, 256, 0, 1, false>", 131072), 13: ("k_hop_p<double, 0, 2, 256, 1, 1, false>", 65536),
    14: ("k_hop_tp<double, 0, 2, 4>", 65536), 15: ("k_hop_tp<double, 0, 2, 8>", 131072),
    16: ("k_hop_ps<double, 0, 2, 256, 1, false>", 65536), 17: ("k_hop_ps<double, 0, 2, 256, 1, false>", 131072),
    18: ("k_hop_ps<double, 0, 2, 128, 1, false>", 65536), 19: ("k_hop_p<double, 0, 2, 256, 0, 2, false>", 131072),
    28: ("k_hop_p<double, 0, 2, 256, 0, 4, true>", 65536), 29: ("k_hop_p<double, 0, 2, 256, 0, 4, true>", 131072),
    30: ("k_hop_px<double, 0, 2, 256, 2, true>", 65536), 31: ("k_hop_px<double, 0, 2, 256, 2, true>", 131072),
    32: ("k_hop_px<double, 0, 2, 128, 2, true>", 65536), 33: ("k_hop_px<double, 0, 2, 256, 4, true>", 65536),
    34: ("k_hop_ps<double, 0, 2, 256, 2, true>", 65536), 35: ("k_hop_ps<double, 0, 2, 128, 2, true>", 65536),
    36: ("k_hop_px<double, 0, 2, 256, 4, true>", 131072), 37: ("k_hop_px<double, 0, 2, 256, 2, true>", 262144),
    40: ("k_hop_px<double, 0, 2, 256, 4, true>", 196608),
}
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hop_fp64_32c64_hbm_traffic.txt")
# the sources the hop kernels are compiled from: the counter summary records their hash, and a
# summary taken from other sources is not used
HOP_SOURCES = ["hop.hip", "hop_kernels.h", "hop_core.h", "dirac_ops.h", "common.h"]


def hop_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for name in HOP_SOURCES:
        with open(os.path.join(ROOT, "paper_2502_02490_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel: str, grid: int):
    """HBM bytes per launch (copy-calibrated FETCH_SIZE + WRITE_SIZE) of `kernel` with `grid`
    work-items from the committed counter summary, or None when the summary is missing, was
    taken from other kernel sources, or has no such row."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    src = [l for l in lines if l.startswith("# kernel sources sha256:")]
    if not src or src[0].split(":", 1)[1].split()[0] != hop_source_hash():
        return None
    for l in lines:
        if l.startswith("#") or "|" not in l:
            continue
        cols = [c.strip() for c in l.split("|")]
        if len(cols) >= 8 and cols[0] == kernel and cols[1] == str(grid):
            return (float(cols[6]) + float(cols[7])) * 1e9
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed(fn, n, stream):
    import torch

    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(n):
        fn()
    stop.record(stream)
    stop.synchronize()
    return start.elapsed_time(stop) / 1e3  # seconds


def _oracle_schur_rate(reps: int):
    """The oracle's D-hat (FP64, numpy, one thread) on a 16^4 lattice with the same parameters and
    field recipe: the same per-site work as the 32^3 x 64 workload on 1/32 of its volume.  As for
    the GPU, the clover field and its inverse are set-up work outside the timed applies.
    Returns (GB/s of algorithmic bytes, seconds per apply)."""
    import gen
    from oracle import dirac as odirac

    dims = (16, 16, 16, 16)
    f = odirac.Fields(gen.su3_field(dims, EPS, SEED), gen.u1_field(dims, 0.3, SEED),
                      odirac.Params(dims, KAPPA, CSW, CSW_QED, QHAT))
    ev, _ = odirac.even_odd(f)
    f.clover()
    f.clover_inv()
    psi_e = gen.gaussian_spinor(dims, SEED)[ev]
    from threadpoolctl import threadpool_limits

    with threadpool_limits(limits=1):
        odirac.apply_schur(f, psi_e)
        t0 = time.perf_counter()
        for _ in range(reps):
            odirac.apply_schur(f, psi_e)
        dt = (time.perf_counter() - t0) / reps
    return len(ev) * SCHUR_REALS * 8 / dt / 1e9, dt


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(reps: int = 20):
    """The oracle's Schur apply timed on this host's cores: one thread, then one single-threaded
    worker process per usable core (at most 16, each on its own copy of the problem, all started
    together), whose summed rate is the all-core figure."""
    import subprocess

    one, dt = _oracle_schur_rate(reps)
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count() or 1
    workers = max(1, min(16, ncpu))
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1", HIP_VISIBLE_DEVICES="")
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", str(max(4, reps // 2))],
                              stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, env=env, text=True)
             for _ in range(workers)]
    rates = []
    for pr in procs:
        out, _ = pr.communicate(timeout=600)
        if pr.returncode == 0 and out.strip():
            rates.append(json.loads(out.strip().splitlines()[-1])["GBps"])
    allc = sum(rates)
    return {"value": round(allc, 4), "unit": "GB/s", "cores": len(rates), "kind": "oracle",
            "sample": f"oracle D-hat (FP64, numpy) on a 16^4 lattice with the 32^3x64 parameters (same per-site "
                      f"work, 1/32 of the volume), clover set-up excluded: {len(rates)} single-threaded processes "
                      f"at once, {max(4, reps // 2)} applies each (summed rate); one thread alone {one:.4f} GB/s "
                      f"({dt:.2f} s per apply, mean of {reps})",
            "single_thread_GBps": round(one, 4), "nproc": ncpu, "cpu_model": _cpu_model()}


# restart of the inner GCR of the mixed solves, per inner precision: the inner solves stop at 1e-5
# (FP32) or 1e-3 (FP16), where a short restart takes the same iterations for fewer orthogonalisation
# bytes (32^3x64: FP32 0.045 s with GCR(8) against 0.057 s with GCR(32)); the BF16 inner solves stop
# at 1e-2 within a few iterations, where the restart makes no difference
MIXED_INNER_RESTART = {"f32": 8, "f16": 8, "bf16": 32}


def solve_suite(D, b, inner_precs):
    """Time to |b - D x| / |b| < 1e-10: plain FP64 even-odd GCR(32), then FP64 defect correction
    around FP32 / FP16 / BF16 inner GCR (restart MIXED_INNER_RESTART); each mixed solution is
    compared with the FP64 one."""
    import torch

    import paper_2502_02490_amd as P

    res = {}
    # untimed loose solves first: the launch-shape tuner times its candidates on the first call
    # of each kernel at a new lattice size and precision, which must not land in the timings
    for kw in (dict(method=P.GCR, restart=32),) + tuple(dict(method=P.MIXED_GCR, inner_prec=pr,
                                                             restart=MIXED_INNER_RESTART[pr]) for pr in inner_precs):
        D.solve(torch.zeros_like(b), b, tol=1e-4, max_iter=100000, **kw)
    x64 = torch.zeros_like(b)
    info = D.solve(x64, b, method=P.GCR, tol=1e-10, restart=32, max_iter=100000)
    res["fp64_gcr"] = {"seconds": round(info.seconds, 4), "iters": info.iters, "restarts": info.restarts,
                       "true_rel_res": info.true_rel_res}
    nx = torch.linalg.vector_norm(x64).item()
    for pr in inner_precs:
        x = torch.zeros_like(b)
        info = D.solve(x, b, method=P.MIXED_GCR, inner_prec=pr, tol=1e-10, restart=MIXED_INNER_RESTART[pr],
                       max_iter=100000)
        res[f"mixed_{pr}"] = {"seconds": round(info.seconds, 4), "inner_restart": MIXED_INNER_RESTART[pr],
                              "inner_iters": info.iters, "outer": info.outer,
                              "fell_back": info.fell_back, "true_rel_res": info.true_rel_res,
                              "rel_err_vs_fp64": torch.linalg.vector_norm(x - x64).item() / nx,
                              "speedup_vs_fp64": round(res["fp64_gcr"]["seconds"] / info.seconds, 3)}
    return res


# algorithmic bytes per site and Schwarz step of one colour (FP32): the residual, the solution and
# the correction (read / written once: 5 x 96), the corrections of the face neighbours and their
# links (on average 2 of the 8 directions cross a face of a 4^4 block: 2 x (96 + 52)), the clover
# field (288) and the forward links of the hops inside the block (3 of 4 directions: 3 x 52), both
# once per block solve (held in registers and LDS over its minimal-residual steps, whatever their
# number); a site takes one step per cycle
def sap_bytes_per_site(ncy, nmr):
    # per cycle (each site in one colour step): residual read and written, solution read and
    # written, correction written, the face neighbours' corrections and links, clover block and
    # in-block links; the first cycle reads no solution (it starts at zero)
    return ncy * (5 * 96 + 2 * (96 + 52) + 288 + 3 * 52) - 96


SAP_SETTINGS = ((2, 4), (4, 4), (4, 6))


def sap_suite(D, b, plain_seconds, plain_iters):
    """SAP-preconditioned flexible GCR(32) on the full D to 1e-10 (FP32 Schwarz cycles on 4^4
    blocks) against plain FP64 even-odd GCR(32); and one preconditioner application alone."""
    import torch

    import paper_2502_02490_amd as P

    res = {}
    stream = torch.cuda.current_stream()
    V = math.prod(DIMS)
    r32 = D.to_native(b.to(torch.complex64), "f32", "lex")
    o32 = torch.empty_like(r32)
    for ncy, nmr in SAP_SETTINGS:
        D.sap(o32, r32, ncy, nmr)
        t = timed(lambda: D.sap(o32, r32, ncy, nmr), 10, stream) / 10
        D.solve(torch.zeros_like(b), b, method=P.FGCR_SAP, tol=1e-4, sap_ncy=ncy, sap_nmr=nmr)  # warm-up
        x = torch.zeros_like(b)
        info = D.solve(x, b, method=P.FGCR_SAP, tol=1e-10, sap_ncy=ncy, sap_nmr=nmr, max_iter=100000)
        res[f"ncy{ncy}_nmr{nmr}"] = {
            "seconds": round(info.seconds, 4), "iters": info.iters, "fell_back": info.fell_back,
            "true_rel_res": info.true_rel_res, "speedup_vs_fp64_eo_gcr": round(plain_seconds / info.seconds, 3),
            "iters_plain": plain_iters, "precond_ms": round(t * 1e3, 3),
            "precond_algorithmic_GBps": round(sap_bytes_per_site(ncy, nmr) * V / t / 1e9, 1)}
    return res


def sap_kernels(reps: int):
    """The Schwarz preconditioner alone on 32^3 x 64 (the benchmark field): one application with
    4 cycles of 4 minimal-residual steps, timed with HIP events; one JSON line."""
    import torch

    import gen
    import paper_2502_02490_amd as P

    D = P.Dirac(torch.from_numpy(gen.su3_field(DIMS, EPS, SEED)).cuda(), torch.from_numpy(gen.u1_field(DIMS, 0.3, SEED)).cuda(),
                DIMS, KAPPA, CSW, CSW_QED, QHAT)
    r32 = D.to_native(torch.from_numpy(gen.gaussian_spinor(DIMS, SEED)).cuda().to(torch.complex64), "f32", "lex")
    o32 = torch.empty_like(r32)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        D.sap(o32, r32, 4, 4)
    t = timed(lambda: D.sap(o32, r32, 4, 4), reps, stream) / reps
    V = math.prod(DIMS)
    out = {"lattice": "x".join(map(str, DIMS)), "ncy": 4, "nmr": 4, "precond_ms": round(t * 1e3, 3),
           "bytes_per_site": sap_bytes_per_site(4, 4),
           "algorithmic_GBps": round(sap_bytes_per_site(4, 4) * V / t / 1e9, 1),
           "frac_of_8TBps": round(sap_bytes_per_site(4, 4) * V / t / 8e12, 3)}
    D.close()
    return out


BATCH_DIMS = [(8, 8, 8, 8), (12, 12, 12, 12)] + [(32, 16, 16, 16)] * 3 + [(48, 24, 24, 24)] * 3
# restart of the batched inner FP32 GCR: the inner solves stop at 1e-5, where GCR(8) takes about the
# iterations GCR(32) does at a quarter of the orthogonalisation bytes (measured 0.39 s against 0.54 s)
BATCH_INNER_RESTART = 8


def batched_suite():
    """12 spin-colour point sources (at the origin) on each of 8 lattices of uneven size, kappa_j =
    0.120 + 0.005 j / 7, eps = 0.5, c_sw = 1.6, c_sw^QED = 1.0, qhat = -1, seeds 401 + j; FP64
    defect correction around batched FP32 GCR(8), to 1e-10; compared with the 96 plain FP64
    even-odd GCR(32) solves and the 96 same mixed solves done one after another on the same GPU."""
    import numpy as np
    import torch

    import gen
    import paper_2502_02490_amd as P

    ops, bs = [], []
    for j, d in enumerate(BATCH_DIMS):
        U = gen.su3_field(d, EPS, 401 + j)
        th = gen.u1_field(d, 0.3, 401 + j)
        ops.append(P.Dirac(torch.from_numpy(U).cuda(), torch.from_numpy(th).cuda(), d, 0.120 + 0.005 * j / 7, CSW,
                           CSW_QED, QHAT))
        V = math.prod(d)
        b = torch.zeros((12, V, 4, 3), dtype=torch.complex128, device="cuda")
        for s_ in range(4):
            for a in range(3):
                b[3 * s_ + a, 0, s_, a] = 1.0
        bs.append(b)
    xs = [torch.zeros_like(b) for b in bs]
    P.solve_batched(ops, xs, bs, 12, method=P.MIXED_GCR, inner_prec="f32", tol=1e-10,
                    restart=BATCH_INNER_RESTART)  # tuning, graphs
    xs = [torch.zeros_like(b) for b in bs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = P.solve_batched(ops, xs, bs, 12, method=P.MIXED_GCR, inner_prec="f32", tol=1e-10,
                            restart=BATCH_INNER_RESTART)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    t1 = time.perf_counter()
    err, iters = 0.0, 0
    for D, b, x in zip(ops, bs, xs):
        for r in range(12):
            y = torch.zeros_like(b[r])
            inf = D.solve(y, b[r].contiguous(), method=P.GCR, tol=1e-10, restart=32)
            iters += inf.iters
            err = max(err, (torch.linalg.vector_norm(x[r] - y) / torch.linalg.vector_norm(y)).item())
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t1
    # the same mixed-precision solves one right-hand side at a time (what batching saves)
    t2 = time.perf_counter()
    for D, b in zip(ops, bs):
        for r in range(12):
            y = torch.zeros_like(b[r])
            D.solve(y, b[r].contiguous(), method=P.MIXED_GCR, inner_prec="f32", tol=1e-10, restart=BATCH_INNER_RESTART)
    torch.cuda.synchronize()
    t_seq_mixed = time.perf_counter() - t2
    worst = max(i.true_rel_res for row in infos for i in row)
    # the same batch with BF16 inner solves (GCR(16) inside), which the mixed scheme also offers
    xb = [torch.zeros_like(b) for b in bs]
    P.solve_batched(ops, xb, bs, 12, method=P.MIXED_GCR, inner_prec="bf16", tol=1e-10, restart=16)
    xb = [torch.zeros_like(b) for b in bs]
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    infb = P.solve_batched(ops, xb, bs, 12, method=P.MIXED_GCR, inner_prec="bf16", tol=1e-10, restart=16)
    torch.cuda.synchronize()
    t_bf16 = time.perf_counter() - t3
    worst_bf16 = max(i.true_rel_res for row in infb for i in row)
    diff_bf16 = max((torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item()
                    for xa, xf in zip(xb, xs) for a, b in zip(xa, xf))
    del xb
    for D in ops:
        D.close()
    return {"lattices": ["x".join(map(str, d)) for d in BATCH_DIMS], "nrhs": 12, "inner_restart": BATCH_INNER_RESTART,
            "batched_mixed_f32_seconds": round(t_batched, 4), "sequential_fp64_gcr_seconds": round(t_seq, 4),
            "speedup_vs_sequential_fp64": round(t_seq / t_batched, 3),
            "sequential_mixed_f32_seconds": round(t_seq_mixed, 4),
            "speedup_vs_sequential_mixed_f32": round(t_seq_mixed / t_batched, 3), "worst_true_rel_res": worst,
            "max_rel_diff_vs_fp64": err, "fp64_total_iters": iters,
            "batched_mixed_bf16_seconds": round(t_bf16, 4), "batched_mixed_bf16_worst_true_rel_res": worst_bf16,
            "batched_mixed_bf16_max_rel_diff_vs_f32": diff_bf16,
            "batched_mixed_bf16_speedup_vs_sequential_fp64": round(t_seq / t_bf16, 3),
            "inner_iters_per_lattice": [max(i.iters for i in row) for row in infos],
            "host_syncs": infos[0][0].host_syncs}


PTC_TRAIN_DIMS = (32, 16, 16, 16)
PTC_KAPPA = 0.1245
# algorithmic bytes of one network application per site, layer by layer (each activation read
# once and written once in FP32, links as 13 FP32 reals per direction): 1 -> 8: 96 + 768 + 416,
# 8 -> 8: 768 + 768 + 416, 8 -> 1: 768 + 96 + 416
PTC_BYTES_PER_SITE = 1280 + 1952 + 1280


def local_share(extra, steps, stream):
    """The Schur apply on 48^3 x 12, one GPU's share of 48^3 x 96 cut along t over 8 GPUs (same
    parameters, periodic in every direction here; the halo exchange itself is not built)."""
    import numpy as np
    import torch

    import gen
    import paper_2502_02490_amd as P

    local = (12, 48, 48, 48)
    vhl = math.prod(local) // 2
    Dl = P.Dirac(torch.from_numpy(gen.su3_field(local, EPS, SEED)).cuda(),
                 torch.from_numpy(gen.u1_field(local, 0.3, SEED)).cuda(), local, KAPPA, CSW, CSW_QED, QHAT)
    psi_l = gen.gaussian_spinor(local, SEED)
    for pr in ("f64", "f32"):
        src = psi_l if pr == "f64" else psi_l.astype(np.complex64)
        xe_l = Dl.to_native(torch.from_numpy(src).cuda(), pr, "lex")
        xe_l = xe_l[: xe_l.numel() // 2].clone()
        ye_l = torch.empty_like(xe_l)
        sl = lambda: Dl.apply_eo(ye_l, xe_l, pr, "native")  # noqa: E731
        for _ in range(5):
            sl()
        tl = timed(sl, steps, stream)
        extra[f"schur_{pr}_local_48c12_GBps"] = round(SCHUR_REALS * (8 if pr == "f64" else 4) * vhl * steps / tl / 1e9, 1)
        extra[f"schur_{pr}_local_48c12_us"] = round(tl / steps * 1e6, 1)
    Dl.close()
    del Dl, xe_l, ye_l


def gcr_solves(n: int):
    """n plain FP64 even-odd GCR(32) solves to 1e-10 on the bench's 32^3x64 field and source (the
    first one also tunes the launch shapes)."""
    import torch

    import gen
    import paper_2502_02490_amd as P

    D = P.Dirac(torch.from_numpy(gen.su3_field(DIMS, EPS, SEED)).cuda(), torch.from_numpy(gen.u1_field(DIMS, 0.3, SEED)).cuda(),
                DIMS, KAPPA, CSW, CSW_QED, QHAT)
    b = torch.from_numpy(gen.gaussian_spinor(DIMS, SEED)).cuda()
    out = []
    for _ in range(n):
        x = torch.zeros_like(b)
        info = D.solve(x, b, method=P.GCR, tol=1e-10, restart=32, max_iter=100000)
        out.append({"iters": info.iters, "seconds": round(info.seconds, 4), "true_rel_res": info.true_rel_res})
    D.close()
    return {"lattice": "x".join(map(str, DIMS)), "solves": out}


def copy_calibration(n: int = 5):
    """n plain device copies of exactly 768 MiB (read and written): a kernel of known size that
    scales the FETCH_SIZE / WRITE_SIZE counters of a profiled run."""
    import torch

    src = torch.ones(768 * 2**20 // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(n):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def apply_kernels(reps: int):
    """The Schur applies alone on the 32^3 x 64 workload, in each storage precision, and the FP32
    apply of 12 right-hand sides in one call; each timed with HIP events after the tuner has
    picked its launch shapes.  One JSON line (for kernel traces and counter runs)."""
    import numpy as np
    import torch

    import gen
    import paper_2502_02490_amd as P

    D = P.Dirac(torch.from_numpy(gen.su3_field(DIMS, EPS, SEED)).cuda(),
                torch.from_numpy(gen.u1_field(DIMS, 0.3, SEED)).cuda(), DIMS, KAPPA, CSW, CSW_QED, QHAT)
    psi = torch.from_numpy(gen.gaussian_spinor(DIMS, SEED)).cuda()
    stream = torch.cuda.current_stream()
    vh = math.prod(DIMS) // 2
    out = {"lattice": "x".join(map(str, DIMS))}
    for pr, rb in (("f64", 8), ("f32", 4), ("f16", 2), ("bf16", 2)):
        src = psi.to(torch.complex64) if pr == "f32" else psi
        x = D.to_native(src, pr, "lex")
        xe = x[: x.numel() // 2].clone()
        ye = torch.empty_like(xe)
        fn = lambda: D.apply_eo(ye, xe, pr, "native")  # noqa: E731
        for _ in range(3):
            fn()
        t = timed(fn, reps, stream) / reps
        out[f"schur_{pr}_us"] = round(t * 1e6, 1)
        out[f"schur_{pr}_GBps"] = round(SCHUR_REALS * rb * vh / t / 1e9, 1)
        if pr == "f32":
            nr = 12
            x12 = torch.cat([xe] * nr)
            y12 = torch.empty_like(x12)
            m12 = lambda: D.apply_eo_multi(y12, x12, nr, "f32")  # noqa: E731
            for _ in range(3):
                m12()
            t12 = timed(m12, reps, stream) / reps
            out["schur_f32_12rhs_us_per_rhs"] = round(t12 / nr * 1e6, 1)
            out["schur_f32_12rhs_GBps"] = round((nr * 120 + 352) * 4 * vh / t12 / 1e9, 1)
            del x12, y12
        del x, xe, ye
    D.close()
    return out


def ptc_kernels(reps: int):
    """The network's kernels alone on 32^3 x 64 (seed 505 field, seed-7 initial weights): one
    forward application, one even-odd application (the Schur-system preconditioner: even half in,
    even half out) and one backward pass (forward with every activation kept, weight and input
    gradients), timed with HIP events; one JSON line."""
    import torch

    import gen
    import paper_2502_02490_amd as P
    from paper_2502_02490_amd import ptc_train as T

    d = DIMS
    D = P.Dirac(torch.from_numpy(gen.su3_field(d, EPS, 505)).cuda(), torch.from_numpy(gen.u1_field(d, 0.3, 505)).cuda(),
                d, PTC_KAPPA, CSW, CSW_QED, QHAT)
    net = P.PTC((1, 8, 8, 1))
    net.set_weights(T.init_weights((1, 8, 8, 1), seed=7))
    vin = D.to_native(torch.from_numpy(gen.gaussian_spinor(d, 505)).cuda().to(torch.complex64), "f32", "lex")
    g = D.to_native(torch.from_numpy(gen.gaussian_spinor(d, 506)).cuda().to(torch.complex64), "f32", "lex")
    vout, gin = torch.empty_like(vin), torch.empty_like(vin)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        net.forward(D, vout, vin)
        net.backward(D, gin, vin, g)
    t_f = timed(lambda: net.forward(D, vout, vin), reps, stream) / reps
    half = vin.numel() // 2
    vin_e, vout_e = vin[:half].clone(), torch.empty_like(vin[:half])
    net.forward_eo(D, vout_e, vin_e)
    t_eo = timed(lambda: net.forward_eo(D, vout_e, vin_e), reps, stream) / reps
    t_b = timed(lambda: net.backward(D, gin, vin, g), max(1, reps // 4), stream) / max(1, reps // 4)
    V = math.prod(d)
    out = {"lattice": "x".join(map(str, d)), "channels": [1, 8, 8, 1],
           "forward_ms": round(t_f * 1e3, 3), "forward_eo_ms": round(t_eo * 1e3, 3),
           "backward_ms": round(t_b * 1e3, 3),
           "forward_algorithmic_GBps": round(PTC_BYTES_PER_SITE * V / t_f / 1e9, 1),
           "forward_frac_of_8TBps": round(PTC_BYTES_PER_SITE * V / t_f / 8e12, 3),
           "forward_contraction_TFLOPs": round(ptc_flop_per_site((1, 8, 8, 1)) * V / t_f / 1e12, 1)}
    D.close()
    net.close()
    return out


# networks trained and deployed by the learned-preconditioner suite: the configured (1, 8, 8, 1)
# and two thin ones, all on the same pairs; the suite reports each and selects the one with the
# shortest measured time to solution
PTC_NETWORKS = ((1, 8, 8, 1), (1, 4, 1), (1, 2, 2, 2, 1))
PTC_TRAIN_BUDGET_S = {(1, 8, 8, 1): 40.0, (1, 4, 1): 15.0, (1, 2, 2, 2, 1): 20.0}


def ptc_flop_per_site(channels) -> int:
    """Spin contractions of a network per site: 9 paths x c_in x c_out x 16 spin entries x 3
    colours complex multiply-adds (8 real flops each)."""
    return 8 * 9 * 16 * 3 * sum(a * b for a, b in zip(channels[:-1], channels[1:]))


def ptc_suite(pairs_per_field: int, epochs: int, checkpoint: str | None):
    """Learned preconditioner: PTC networks (the configured (1, 8, 8, 1) and the thin (1, 4, 1) and
    (1, 2, 2, 2, 1)) trained on the same pairs from four 16^3 x 32 fields (seeds 501..504,
    eps = 0.5, kappa = 0.1245, c_sw = 1.6, c_sw^QED = 1.0, qhat = -1), then each deployed in
    flexible GCR(8) on a 32^3 x 64 field (seed 505) against plain FP64 even-odd GCR(32), all to 1e-10.
    Pair generation and training time are reported apart from the solves; the network with the
    shortest measured solve is the selected one."""
    import torch

    import gen
    import paper_2502_02490_amd as P
    from paper_2502_02490_amd import ptc_train as T

    res = {"train_lattice": "x".join(map(str, PTC_TRAIN_DIMS)), "fields": 4}
    ops_pairs, held = [], []
    t0 = time.perf_counter()
    for j in range(4):
        d = PTC_TRAIN_DIMS
        D = P.Dirac(torch.from_numpy(gen.su3_field(d, EPS, 501 + j)).cuda(),
                    torch.from_numpy(gen.u1_field(d, 0.3, 501 + j)).cuda(), d, PTC_KAPPA, CSW, CSW_QED, QHAT)
        # half from truncated FP64 solves (low-mode dominated errors), half e ~ Gaussian with
        # r = D e (high-mode dominated): both are exact (r, D^-1 r) pairs
        rs, es = T.generate_pairs(D, pairs_per_field // 2, seed=501 + j, log=log)
        ra, ea = T.generate_apply_pairs(D, pairs_per_field - pairs_per_field // 2, seed=601 + j)
        ops_pairs.append((D, rs + ra, es + ea))
        hr, he = T.generate_pairs(D, 6, seed=10501 + j)
        har, hae = T.generate_apply_pairs(D, 6, seed=10601 + j)
        held.append((D, hr + har, he + hae))
        log(f"[ptc] field {j}: {len(rs)} pairs ({time.perf_counter() - t0:.1f} s)")
    res["pairs"] = sum(len(rs) for _, rs, _ in ops_pairs)
    res["pair_kinds"] = "half truncated FP64 GCR solves (e = x* - x_k), half Gaussian e with r = D e"
    res["pair_generation_seconds"] = round(time.perf_counter() - t0, 2)
    nets, per = {}, {}
    for ch in PTC_NETWORKS:
        key = "-".join(map(str, ch))
        net = P.PTC(ch)
        net.set_weights(T.init_weights(ch, seed=7))
        r = {"channels": list(ch), "held_out_loss_init": T.evaluate(held, net)}
        t1 = time.perf_counter()
        hist = T.train(ops_pairs, net, epochs=epochs, batch=16, lr=2e-3, seed=11, lr_decay=0.8,
                       log=lambda m: log(f"[ptc {key}] " + m), time_budget=PTC_TRAIN_BUDGET_S[ch])
        r["training_seconds"] = round(time.perf_counter() - t1, 2)
        r["train_loss_by_epoch"] = [round(h, 5) for h in hist]
        r["held_out_loss"] = T.evaluate(held, net)
        log(f"[ptc {key}] held-out loss {r['held_out_loss_init']:.4f} -> {r['held_out_loss']:.4f}")
        if checkpoint and ch == PTC_NETWORKS[0]:
            T.save_checkpoint(checkpoint, net, len(hist), 11, meta={"pairs": res["pairs"], "train": res["train_lattice"]})
        nets[key], per[key] = net, r
    for D, _, _ in ops_pairs:
        D.close()
    del ops_pairs, held
    torch.cuda.empty_cache()
    d = DIMS
    D = P.Dirac(torch.from_numpy(gen.su3_field(d, EPS, 505)).cuda(), torch.from_numpy(gen.u1_field(d, 0.3, 505)).cuda(),
                d, PTC_KAPPA, CSW, CSW_QED, QHAT)
    b = torch.from_numpy(gen.gaussian_spinor(d, 505)).cuda()
    vin = D.to_native(b.to(torch.complex64), "f32", "lex")
    vout = torch.empty_like(vin)
    stream = torch.cuda.current_stream()
    for key, net in nets.items():
        r = per[key]
        # one network application on 32^3 x 64: the layers on the matrix cores
        for _ in range(3):
            net.forward(D, vout, vin)
        t_fwd = timed(lambda: net.forward(D, vout, vin), 10, stream) / 10
        flop = ptc_flop_per_site(net.channels) * math.prod(d)
        r["forward_32c64_ms"] = round(t_fwd * 1e3, 3)
        r["forward_32c64_contraction_TFLOPs"] = round(flop / t_fwd / 1e12, 1)
        log(f"[ptc {key}] forward 32^3x64: {t_fwd * 1e3:.2f} ms, {flop / t_fwd / 1e12:.1f} TFLOP/s in the spin "
            "contractions")
        T.compare_solvers(D, net, b, tol=1e-10)  # warm-up (tuning, work buffers)
        dep = T.compare_solvers(D, net, b, tol=1e-10, reps=2)
        r["deploy_32c64"] = dep
        for k in ("fgcr_ptc", "fgcr_ptc_eo"):
            r[f"{k}_speedup_vs_eo_gcr"] = round(dep["eo_gcr"]["seconds"] / dep[k]["seconds"], 3)
        log(f"[ptc {key}] deploy {dep}")
    del vin, vout
    best = min(per, key=lambda k: per[k]["deploy_32c64"]["fgcr_ptc_eo"]["seconds"])
    res["networks"] = per
    res["selected"] = best
    res["selected_fgcr_ptc_eo_seconds"] = per[best]["deploy_32c64"]["fgcr_ptc_eo"]["seconds"]
    res["selected_fgcr_ptc_eo_iters"] = per[best]["deploy_32c64"]["fgcr_ptc_eo"]["iters"]
    res["eo_gcr_seconds"] = per[best]["deploy_32c64"]["eo_gcr"]["seconds"]
    res["eo_gcr_iters"] = per[best]["deploy_32c64"]["eo_gcr"]["iters"]
    res["selected_speedup_vs_eo_gcr"] = per[best]["fgcr_ptc_eo_speedup_vs_eo_gcr"]
    D.close()
    for net in nets.values():
        net.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true", help="skip the solve timings")
    ap.add_argument("--no-48", action="store_true", help="skip the 48^3x96 mixed-precision solves")
    ap.add_argument("--no-batched", action="store_true", help="skip the 8-lattice x 12-RHS batched solve")
    ap.add_argument("--no-ptc", action="store_true",
                    help="skip the learned preconditioner (trained on 16^3x32 pairs, deployed on 32^3x64)")
    ap.add_argument("--ptc-pairs", type=int, default=500, help="training pairs per 16^3x32 field")
    ap.add_argument("--ptc-epochs", type=int, default=8)
    ap.add_argument("--ptc-checkpoint", default=None, help="write the trained weights and Adam state here")
    ap.add_argument("--sap-kernels", action="store_true",
                    help="only time the Schwarz preconditioner (4 cycles x 4 block steps) on 32^3x64 (one JSON line)")
    ap.add_argument("--ptc-kernels", action="store_true",
                    help="only time the PTC network's forward and backward kernels on 32^3x64 (one JSON line)")
    ap.add_argument("--no-local", action="store_true",
                    help="skip the Schur apply on 48^3x12 (for counter runs that average per kernel over one lattice)")
    ap.add_argument("--apply-kernels", action="store_true",
                    help="only time the Schur applies on 32^3x64 in FP64 / FP32 / FP16 / BF16 and the FP32 12-RHS apply "
                         "(one JSON line), for kernel traces and counter runs")
    ap.add_argument("--batched-solves", action="store_true",
                    help="only run the 8-lattice x 12 point-source batched solve suite (one JSON line), for a "
                         "kernel trace of the batched iteration")
    ap.add_argument("--gcr-solves", action="store_true",
                    help="only run three plain FP64 even-odd GCR(32) solves on 32^3x64 (one JSON line), for a "
                         "kernel trace of the Krylov BLAS")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run 5 plain device copies of 768 MiB (a known-size kernel for HBM counter calibration)")
    ap.add_argument("--cpu-worker", type=int, default=0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker:
        # one single-threaded worker of the all-core CPU baseline (started by cpu_baseline)
        gbs, dt = _oracle_schur_rate(args.cpu_worker)
        print(json.dumps({"GBps": gbs, "seconds_per_apply": dt}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the operator runs on a single MI355X (multi-GPU halo exchange is "
              "designed, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.sap_kernels:
        import torch

        torch.cuda.set_device(0)
        print(json.dumps({"sap_kernels": sap_kernels(max(1, args.steps // 10))}), flush=True)
        return
    if args.ptc_kernels:
        import torch

        torch.cuda.set_device(0)
        print(json.dumps({"ptc_kernels": ptc_kernels(max(1, args.steps // 10))}), flush=True)
        return
    if args.apply_kernels:
        import torch

        torch.cuda.set_device(0)
        out = apply_kernels(max(1, args.steps))
        if args.copy_calibration:
            copy_calibration()
        print(json.dumps({"apply_kernels": out}), flush=True)
        return
    if args.batched_solves:
        import torch

        torch.cuda.set_device(0)
        print(json.dumps({"batched_solves": batched_suite()}), flush=True)
        return
    if args.gcr_solves:
        import torch

        torch.cuda.set_device(0)
        print(json.dumps({"gcr_solves": gcr_solves(3)}), flush=True)
        return

    # the launch-shape tuner records its choices here, so the line can name the kernel it timed
    tune_cache = os.path.join("/tmp", f"dirac_tune_{os.getpid()}.json")
    os.environ.setdefault("DIRAC_TUNE_CACHE", tune_cache)

    import numpy as np
    import torch

    import gen
    import paper_2502_02490_amd as P

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    U = gen.su3_field(DIMS, EPS, SEED)
    th = gen.u1_field(DIMS, 0.3, SEED)
    psi = gen.gaussian_spinor(DIMS, SEED)
    log(f"[bench] fields generated in {time.perf_counter() - t0:.1f} s")
    V = math.prod(DIMS)
    vh = V // 2
    D = P.Dirac(torch.from_numpy(U).cuda(), torch.from_numpy(th).cuda(), DIMS, KAPPA, CSW, CSW_QED, QHAT)
    x = D.to_native(torch.from_numpy(psi).cuda(), "f64", "lex")
    xe = x[: x.numel() // 2].clone()
    ye = torch.empty_like(xe)
    y = torch.empty_like(x)
    torch.cuda.synchronize()

    # a plain device copy of exactly 768 MiB read + 768 MiB written per launch: its rate is the
    # practical ceiling of a streaming kernel, and in a profiled run (--copy-calibration, five
    # copies) it scales the FETCH_SIZE / WRITE_SIZE counters
    src = torch.ones(768 * 2**20 // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ncopy = 5 if args.copy_calibration else 10
    t_copy = timed(lambda: dst.copy_(src), ncopy, stream)
    copy_gbs = 2 * src.numel() * 8 * ncopy / t_copy / 1e9
    log(f"[bench] device copy 768 MiB: {copy_gbs:.0f} GB/s (read + write)")
    del src, dst
    torch.cuda.synchronize()

    # ---- timed region: K Schur applies (FP64, NATIVE)
    schur = lambda: D.apply_eo(ye, xe, "f64", "native")  # noqa: E731
    for _ in range(args.warmup):
        schur()
    torch.cuda.synchronize()
    t_schur = timed(schur, args.steps, stream)
    torch.cuda.synchronize()
    ms = t_schur / args.steps * 1e3
    gbs = SCHUR_REALS * 8 * vh * args.steps / t_schur / 1e9
    log(f"[bench] Schur FP64: {ms * 1e3:.1f} us/apply, {gbs:.0f} GB/s")

    # ---- dominant kernel alone: the hop + A chi kernel, two launches per full-D apply
    full = lambda: D.apply(y, x, "f64", "native")  # noqa: E731
    for _ in range(5):
        full()
    t_full = timed(full, args.steps, stream)
    k_dur = t_full / (2 * args.steps)
    k_gbs = CLOV_HOP_REALS * 8 * vh / k_dur / 1e9
    log(f"[bench] hop+clover kernel FP64: {k_dur * 1e6:.1f} us/launch, {k_gbs:.0f} GB/s")

    extra = {}
    chosen = None
    try:
        with open(os.environ["DIRAC_TUNE_CACHE"]) as fh:
            choices = json.load(fh)
        key = "hop-v2|f64|dag0|mode2|" + "x".join(map(str, DIMS)) + "|nrhs1|gfx950"
        chosen = int(choices[key])
        extra["tuned_hop_shapes"] = {k.split("|", 1)[1].rsplit("|", 1)[0]: HOP_SHAPES[v] for k, v in choices.items()
                                     if k.startswith("hop-v2|") and "x".join(map(str, DIMS)) in k}
    except (OSError, KeyError, ValueError) as e:
        log(f"[bench] tuner choice not readable: {e}")
    # every launch shape of the hop kernel, FP64 Schur (the tuner's choice is what the timed loop used)
    shapes = {}
    for shape in range(len(HOP_SHAPES)):
        os.environ["DIRAC_HOP_SHAPE"] = str(shape)
        for _ in range(3):
            schur()
        ts = timed(schur, max(10, args.steps // 4), stream)
        shapes[shape] = round(SCHUR_REALS * 8 * vh * max(10, args.steps // 4) / ts / 1e9, 1)
    del os.environ["DIRAC_HOP_SHAPE"]
    extra["schur_f64_GBps_by_shape"] = shapes
    log(f"[bench] Schur FP64 GB/s by launch shape {shapes}")
    # FP32 Schur
    x32 = D.to_native(torch.from_numpy(psi.astype(np.complex64)).cuda(), "f32", "lex")
    xe32 = x32[: x32.numel() // 2].clone()
    ye32 = torch.empty_like(xe32)
    s32 = lambda: D.apply_eo(ye32, xe32, "f32", "native")  # noqa: E731
    for _ in range(5):
        s32()
    t32 = timed(s32, args.steps, stream)
    extra["schur_f32_GBps"] = round(SCHUR_REALS * 4 * vh * args.steps / t32 / 1e9, 1)
    extra["schur_f32_us"] = round(t32 / args.steps * 1e6, 1)
    for pr in ("f16", "bf16"):
        xh = D.to_native(torch.from_numpy(psi).cuda(), pr, "lex")
        xeh = xh[: xh.numel() // 2].clone()
        yeh = torch.empty_like(xeh)
        sh = lambda: D.apply_eo(yeh, xeh, pr, "native")  # noqa: E731
        for _ in range(5):
            sh()
        th_ = timed(sh, args.steps, stream)
        extra[f"schur_{pr}_GBps"] = round(SCHUR_REALS * 2 * vh * args.steps / th_ / 1e9, 1)
        extra[f"schur_{pr}_us"] = round(th_ / args.steps * 1e6, 1)
    # 12 right-hand sides at once (FP32): links and clover read once per site block for all of
    # them; algorithmic bytes per even site 12 x 120 spinor reals + 208 link + 144 clover reals
    nr = 12
    x12 = torch.cat([xe32] * nr)
    y12 = torch.empty_like(x12)
    m12 = lambda: D.apply_eo_multi(y12, x12, nr, "f32")  # noqa: E731
    for _ in range(3):
        m12()
    t12 = timed(m12, max(10, args.steps // 4), stream) / max(10, args.steps // 4)
    extra["schur_f32_12rhs_us_per_rhs"] = round(t12 / nr * 1e6, 1)
    extra["schur_f32_12rhs_GBps"] = round((nr * 120 + 352) * 4 * vh / t12 / 1e9, 1)
    extra["schur_f32_12rhs_speedup_per_rhs"] = round(extra["schur_f32_us"] / extra["schur_f32_12rhs_us_per_rhs"], 2)
    by_shape = {}
    for shape in range(len(HOP_SHAPES)):
        os.environ["DIRAC_HOP_SHAPE"] = str(shape)
        m12()
        by_shape[shape] = round(timed(m12, 10, stream) / 10 / nr * 1e6, 1)
    del os.environ["DIRAC_HOP_SHAPE"]
    extra["schur_f32_12rhs_us_per_rhs_by_shape"] = by_shape
    del x12, y12
    # standalone hop and clover (FP64)
    ho = torch.empty_like(xe)
    hop = lambda: D.apply_hop(ho, xe, 1, "f64")  # noqa: E731
    for _ in range(5):
        hop()
    th_ = timed(hop, args.steps, stream)
    extra["hop_f64_GBps"] = round(152 * 8 * vh * args.steps / th_ / 1e9, 1)
    cl = lambda: D.apply_clover(ho, xe, 0, False, "f64")  # noqa: E731
    for _ in range(5):
        cl()
    tc = timed(cl, args.steps, stream)
    extra["clover_f64_GBps"] = round(120 * 8 * vh * args.steps / tc / 1e9, 1)
    # C* boundaries in directions 1..3 on the same field, read as the doubled lattice (dims[1] = 32
    # holds the physical x extent 16 and its mirror copy): the shifted neighbours cost nothing
    Dc = P.Dirac(torch.from_numpy(U).cuda(), torch.from_numpy(th).cuda(), DIMS, KAPPA, CSW, CSW_QED, QHAT,
                 (math.pi, 0.0, 0.0, 0.0), cstar=3)
    yc = torch.empty_like(xe)
    schur_c = lambda: Dc.apply_eo(yc, xe, "f64", "native")  # noqa: E731
    for _ in range(5):
        schur_c()
    tcs = timed(schur_c, args.steps, stream)
    extra["schur_f64_cstar3_GBps"] = round(SCHUR_REALS * 8 * vh * args.steps / tcs / 1e9, 1)
    Dc.close()
    del Dc
    # one GPU's share of 48^3 x 96 cut along t over 8 GPUs: the Schur apply at 48^3 x 12 (same
    # parameters, periodic in every direction here; the halo exchange itself is not built)
    if not args.no_local:
        local_share(extra, args.steps, stream)
    del yc
    log(f"[bench] extra {extra}")

    solves = {}
    if not args.no_solve:
        solves["32^3x64"] = solve_suite(D, torch.from_numpy(psi).cuda(), ("f32", "f16", "bf16"))
        log(f"[bench] solves 32^3x64 {solves['32^3x64']}")
        plain = solves["32^3x64"]["fp64_gcr"]
        solves["32^3x64_fgcr_sap"] = sap_suite(D, torch.from_numpy(psi).cuda(), plain["seconds"], plain["iters"])
        log(f"[bench] SAP 32^3x64 {solves['32^3x64_fgcr_sap']}")
    D.close()
    del x, xe, ye, y, x32, xe32, ye32
    torch.cuda.empty_cache()
    if not args.no_solve and not args.no_48:
        d3 = (96, 48, 48, 48)
        t0 = time.perf_counter()
        U3 = gen.su3_field(d3, EPS, 301)
        th3 = gen.u1_field(d3, 0.3, 301)
        b3 = gen.gaussian_spinor(d3, 301)
        D3 = P.Dirac(torch.from_numpy(U3).cuda(), torch.from_numpy(th3).cuda(), d3, 0.1250, CSW, CSW_QED, 2)
        del U3, th3
        log(f"[bench] 48^3x96 set-up {time.perf_counter() - t0:.1f} s")
        solves["48^3x96"] = solve_suite(D3, torch.from_numpy(b3).cuda(), ("f32", "f16", "bf16"))
        log(f"[bench] solves 48^3x96 {solves['48^3x96']}")
        D3.close()

    if not args.no_solve and not args.no_batched:
        solves["batched_8lat_12rhs"] = batched_suite()
        log(f"[bench] batched {solves['batched_8lat_12rhs']}")

    if not args.no_solve and not args.no_ptc:
        solves["ptc_learned_preconditioner"] = ptc_suite(args.ptc_pairs, args.ptc_epochs, args.ptc_checkpoint)

    traffic = None
    if chosen is not None and DIMS == (64, 32, 32, 32) and chosen in HOP_CLOV_KERNEL_32C64:
        traffic = profiled_traffic(*HOP_CLOV_KERNEL_32C64[chosen])
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline()
        log(f"[bench] cpu baseline {cpu}")

    out = {
        "metric": "Dirac apply GB/s & %HBM roofline (even-odd Schur D-hat, FP64)",
        "value": round(gbs, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "32^3x64 even-odd Schur apply, FP64, NATIVE layout", "lattice": "64x32x32x32",
                   "kappa": KAPPA, "csw": CSW, "csw_qed": CSW_QED, "qhat": QHAT, "eps": EPS},
        "roofline": {"bound": "hbm", "achieved": round(k_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(k_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "hop + A_pp chi, FP64 (" + (HOP_SHAPES[chosen] if chosen is not None else "?") + ")",
                     "bytes_per_launch": CLOV_HOP_REALS * 8 * vh, "us_per_launch": round(k_dur * 1e6, 2),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "traffic_over_algorithmic": (round(traffic / (CLOV_HOP_REALS * 8 * vh), 3)
                                                  if traffic else None)},
        "schur_frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
        "device_copy_GBps": round(copy_gbs, 1),
        "gflops_schur": round(FLOP_SCHUR * vh * args.steps / t_schur / 1e9, 1),
        **extra,
        "solve": solves,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
