"""Benchmark of the batched two-level Schwarz-FGMRES solve on one MI355X.

Default workload: the 2048 x 1536 grid with mixed 96/64-cell cores (713
subdomains: 72 x 72 interior, 100 x 72 edge and 100 x 100 corner extended
subdomains with PML), 16-cell blocks of permittivity in [1, 12], 32 seeded
point sources x 2 wavelengths {1.0, 1.2} = 64 right-hand sides in one
launch, exact subdomain LU (the many-source block-Thomas kernel), FGMRES(30)
to a 1e-6 relative residual, complex64 arithmetic with an FP64 iterate.

A step is one FGMRES(30) restart cycle of all 64 right-hand sides through the
C ABI (nosdd_solve_device, inputs resident in HBM): 30 two-level Schwarz
sweeps (gather across overlaps, every subdomain solve, core scatter,
operator, coarse correction when configured) with their Arnoldi steps, the
cycle's explicit FP64 residual and the iterate update; each step continues
from the previous step's field.  A complete solve to 1e-6 of the same batch
is timed once as well (time_to_tol_ms).

Printed (one JSON line): subdomain solves per second over the timed steps
(one exact local solve of one subdomain for one RHS is one unit), the time
per step, the time to 1e-6, the roofline of the dominant kernel (the batched
subdomain solve, against FP32 MFMA or HBM, whichever it is closer to; HIP
events on the library stream around its launches in one more, profiled
cycle), the operator / residual kernels against HBM on HBM-sized arrays, and
the FP64 oracle timed on a bounded sample on the host.  The fields are
checked against the FP64 oracle by the GPU tests, not here.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time to 1e-6 residual per global solve; subdomain solves/s; % HBM roofline"
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFS = 157.3
PROFILE_PMC = os.path.join(ROOT, "profiles", "bt_solve_blocks512_pmc.txt")
PROFILE_PMC_MULTI = os.path.join(ROOT, "profiles", "bt_solve_multi_uneven2048_pmc.txt")
NN_WEIGHTS = os.path.join(ROOT, "paper_2509_03622_amd", "weights", "fno_c64_m16_l4.bin")


def core_list(w):
    """The workload's cores (cx0, cx1, cy0, cy1) in tile order: its explicit list,
    else the tensor product of core_x and core_y (row-major)."""
    if w.cores is not None:
        return [tuple(c) for c in w.cores]
    xs = np.concatenate([[0], np.cumsum(w.core_x)])
    ys = np.concatenate([[0], np.cumsum(w.core_y)])
    return [(int(xs[tx]), int(xs[tx + 1]), int(ys[ty]), int(ys[ty + 1]))
            for ty in range(len(w.core_y)) for tx in range(len(w.core_x))]


def tile_geometry(w):
    """(lx, ly, core cells) of every extended subdomain, in tile order: each core
    grows by overlap/2 across every side that is not on the global boundary."""
    ext = w.overlap // 2
    out = []
    for (cx0, cx1, cy0, cy1) in core_list(w):
        lx = cx1 - cx0 + (ext if cx0 > 0 else 0) + (ext if cx1 < w.nx else 0)
        ly = cy1 - cy0 + (ext if cy0 > 0 else 0) + (ext if cy1 < w.ny else 0)
        out.append((lx, ly, (cx1 - cx0) * (cy1 - cy0)))
    return out


def describe_cores(w):
    sizes = sorted({(c[1] - c[0], c[3] - c[2]) for c in core_list(w)})
    if w.cores is None:
        return f"{len(w.core_x)}x{len(w.core_y)} of " + "/".join(str(v) for v in sorted(set(w.core_x + w.core_y)))
    return f"{len(w.cores)} listed cores (" + ", ".join(f"{a}x{b}" for a, b in sizes) + ")"


def local_solve_bytes(lx, ly, core):
    """Algorithmic HBM bytes of one exact subdomain solve (one tile, one RHS):
    the 2 nb - 1 symmetric factor blocks M_k (upper triangle in 2 x 2
    sub-blocks, b (b + 2) / 2 complex64 each) streamed by the block
    forward/backward sweeps, the gathered tile input and the core output."""
    b, nb = min(lx, ly), max(lx, ly)
    return 8 * ((2 * nb - 1) * b * (b + 2) // 2 + lx * ly + core)


def kernel_hash():
    """Hash of the subdomain-solve source without its // comments and blank
    lines: a change of code, not of commentary, invalidates the stored counters."""
    with open(os.path.join(ROOT, "paper_2509_03622_amd", "csrc", "btlu.hip"), encoding="utf-8") as f:
        lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in f.read().splitlines()]
    return hashlib.sha256("\n".join(ln for ln in lines if ln).encode()).hexdigest()[:16]


def read_traffic(units_per_launch, multi=False):
    """HBM bytes per launch from the committed rocprofv3 counter summary of the
    kernel, or None when it is missing or was taken on a different version of
    the kernel's source file."""
    path = PROFILE_PMC_MULTI if multi else PROFILE_PMC
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def stencil_roofline(torch, nosdd, n_rhs=16, reps=20):
    """Operator y = A x and residual r = b - A x on HBM-sized arrays (2048 x 1536
    grid, n_rhs vectors of 25 MB each), timed with events on the library stream."""
    from paper_2509_03622_amd.workloads import uneven_2048x1536
    w = uneven_2048x1536()
    N = w.nx * w.ny
    ctx = nosdd.Context(0, nosdd.torch_stream_handle())
    P = nosdd.Problem(ctx, w.eps, w.h, w.npml, [64] * (w.nx // 64), [64] * (w.ny // 64), w.overlap, [1.0])
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn((n_rhs, w.ny, w.nx), dtype=torch.complex64, device="cuda", generator=g)
    b = torch.randn((n_rhs, w.ny, w.nx), dtype=torch.complex64, device="cuda", generator=g)
    y = torch.empty_like(x)
    out = {}
    for name, bb, bytes_per_cell in (("operator", None, 16.0 + 4.0 / n_rhs), ("residual", b, 24.0 + 4.0 / n_rhs)):
        P.apply_operator(x, y, bb, n_rhs)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            P.apply_operator(x, y, bb, n_rhs)
        e1.record()
        torch.cuda.synchronize()
        us = 1e3 * e0.elapsed_time(e1) / reps
        gbs = bytes_per_cell * N * n_rhs / (us * 1e-6) / 1e9
        out[name] = {"avg_launch_us": round(us, 1), "achieved_GBs": round(gbs, 1),
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_cell_per_rhs": round(bytes_per_cell, 3)}
    out["shape"] = f"{w.nx}x{w.ny} x {n_rhs} RHS (complex64), algorithmic bytes: x, b read, y written, eps shared"
    P.close()
    ctx.close()
    return out


def host_cpu():
    """Model name of the host CPU and the number of cores this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_sample(w, max_cells=1 << 20):
    """The workload itself when it has at most max_cells cells, else its
    lower-left 512 x 512 window (same permittivity map, same core widths from
    the lower-left corner, the last core of each axis widened to the window
    edge, which carries its own PML), with the source at the window's centre:
    the same subdomain sizes and PML-bearing subdomains, and a size the oracle
    sets up in seconds."""
    if w.nx * w.ny <= max_cells or w.cores is not None:
        return w, "the workload itself"
    from paper_2509_03622_amd.workloads import Workload

    def axis(cores, n=512):
        out, tot = [], 0
        for c in cores:
            if tot + c > n - cores[-1]:
                break
            out.append(c)
            tot += c
        out.append(n - tot)
        return out
    cx, cy = axis(w.core_x), axis(w.core_y)
    sub = Workload(w.name + "_window512", 512, 512, np.ascontiguousarray(w.eps[:512, :512]), list(w.wavelengths),
                   [(256, 256)], cx, cy, overlap=w.overlap, k_coarse=w.k_coarse, npml=w.npml)
    return sub, f"lower-left 512 x 512 window of the workload's permittivity (cores {cx} x {cy}), source at its centre"


def cpu_baseline(w, iters, direct=True):
    """The FP64 oracle on one wavelength and one source of the workload (or of
    a bounded window of it, cpu_sample): its Schwarz-FGMRES with exact
    sparse-LU subdomain solves (construction and the subdomain factorisations
    excluded), capped at `iters` outer iterations, and, when `direct`, the
    global sparse LU factor + solve (SuperLU, single-threaded) of the same
    problem."""
    w, where = cpu_sample(w)
    try:
        from threadpoolctl import threadpool_limits
        lim = threadpool_limits(1)
    except Exception:
        lim = None
    from oracle.fdfd import solve_direct, source_rhs
    from oracle.fgmres import fgmres
    from oracle.schwarz import SchwarzProblem
    lam = w.wavelengths[0]
    t0 = time.perf_counter()
    P = SchwarzProblem(w.eps, lam, w.h, w.npml, w.core_x, w.core_y, w.overlap, k_coarse=w.k_coarse,
                       k_trial=w.k_trial, cores=w.cores)
    for L in P.locs:
        L.lu                                          # factorise every subdomain (excluded)
    setup_s = time.perf_counter() - t0
    b = source_rhs(w.J()[0], lam)
    t0 = time.perf_counter()
    x, it, hist, res = fgmres(lambda u: P.A @ u, b, P.precond, tol=1e-6, restart=30, max_iters=iters)
    dt = time.perf_counter() - t0
    n_tiles = len(core_list(w))
    out = {"value": n_tiles * it / dt, "unit": "subdomain solves/s", "cores": 1, "kind": "oracle",
           "sample": f"{where}; wavelength {lam}, one source, {it} outer FGMRES iterations of the "
                     f"{'two' if w.k_coarse else 'one'}-level Schwarz preconditioner with exact sparse-LU solves "
                     f"of all {n_tiles} subdomains, {dt:.1f} s; construction and subdomain factorisations "
                     f"({setup_s:.1f} s) excluded",
           "ms_per_iteration": 1e3 * dt / max(it, 1)}
    model, avail = host_cpu()
    out["cpu_model"] = model
    out["host_cores_available"] = avail
    if direct:
        t0 = time.perf_counter()
        solve_direct(P.A, b)
        out["direct_splu_s"] = round(time.perf_counter() - t0, 2)
        out["direct_note"] = "global sparse LU (SuperLU, one thread) factor + solve of the same right-hand side"
    if lim is not None:
        lim.unregister()
    return out


def timed_solve(torch, P, J, E, max_iters, reps=1):
    """One untimed solve, then `reps` timed ones; returns seconds per solve,
    iterations, final residuals, status and per-class kernel ms per solve."""
    P.solve_device(J, E, max_iters=max_iters)
    torch.cuda.synchronize()
    P.profile(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        hist, iters, fin, st = P.solve_device(J, E, max_iters=max_iters)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    P.profile(False)
    ms_k, launches, units = P.kernel_times()
    return dt, iters, fin, st, [round(float(v) / reps, 2) for v in ms_k]


def nn_compare(torch, nosdd, workload, configs, max_iters, weights=NN_WEIGHTS):
    """Time to a 1e-6 residual of the exact-LU form and of the NN-FGMRES form
    (BF16 network inside FP32 inner FGMRES) on the same problem and GPU."""
    from paper_2509_03622_amd.workloads import WORKLOADS
    w = WORKLOADS[workload]()
    dev = torch.device("cuda:0")
    J = torch.from_numpy(w.J()).to(dev)
    E = torch.zeros((len(w.wavelengths), len(w.sources), w.ny, w.nx), dtype=torch.complex64, device=dev)
    ctx = nosdd.Context(0, nosdd.torch_stream_handle())
    rows = []
    for kc, solver, steps, tol in configs:
        P = nosdd.Problem(ctx, w.eps, w.h, w.npml, w.core_x, w.core_y, w.overlap, w.wavelengths, w.pml_m, w.pml_lnR)
        t0 = time.perf_counter()
        if solver == "lu":
            P.setup(k_coarse=kc, k_trial=w.k_trial)
        else:
            P.setup(k_coarse=kc, k_trial=w.k_trial, sub_solver=1, nn_weights=weights, inner_max=steps,
                    inner_tol=tol)
        torch.cuda.synchronize()
        setup_ms = 1e3 * (time.perf_counter() - t0)
        dt, iters, fin, st, ms_k = timed_solve(torch, P, J, E, max_iters)
        row = {"solver": solver, "k_coarse": kc, "inner_max": steps, "inner_tol": tol,
               "time_to_tol_ms": round(1e3 * dt, 2), "outer_iterations": int(iters.ravel()[0]),
               "final_rel_residual": float(f"{float(fin.ravel()[0]):.3e}"), "status": int(st),
               "setup_ms": round(setup_ms, 1),
               "kernel_ms": dict(zip(("local_solve", "operator", "arnoldi", "coarse"), ms_k))}
        rows.append(row)
        print(f"[bench] {row}", file=sys.stderr, flush=True)
        P.close()
    ctx.close()
    return w, rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="uneven2048")
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--max-iters", type=int, default=4000,
                    help="outer iteration cap per solve (a small cap shortens profiling runs; the line then "
                         "reports the solves as not converged)")
    ap.add_argument("--cpu-iters", type=int, default=60,
                    help="outer iterations of the CPU oracle timed for cpu_baseline")
    ap.add_argument("--no-direct", action="store_true", help="cpu_baseline without the global sparse LU")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="accepted for compatibility; fields are checked by the tests")
    ap.add_argument("--no-stencil", action="store_true", help="skip the operator/residual roofline measurement")
    ap.add_argument("--no-full-solve", action="store_true",
                    help="skip the complete solve to 1e-6 (time_to_tol_ms); for profiling runs")
    ap.add_argument("--adjoint", action="store_true",
                    help="instead of the default line: one inverse-design gradient (forward + adjoint solves) on "
                         "the 1024 x 1024, three-wavelength design workload")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (calibration of the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--paper-compare", action="store_true",
                    help="instead of the default line: the paper's Algorithm 3 loop (stationary Robin-data sweeps, "
                         "momentum, Robin-space coarse correction) against the FGMRES form, to 1e-5 on the default "
                         "workload")
    ap.add_argument("--quadtree-compare", action="store_true",
                    help="instead of the default line: the 512 x 512 quad-tree workload (64-cell cores in vacuum, "
                         "32-cell cores over the high-index square) against uniform 64- and 32-cell partitions of "
                         "the same problem, time to 1e-6")
    ap.add_argument("--nn-compare", action="store_true",
                    help="instead of the default line: exact-LU against NN-FGMRES subdomain solves, time to 1e-6 "
                         "on the 1024 x 1024 workload (16 x 16 subdomains)")
    ap.add_argument("--weights", default=NN_WEIGHTS, help="--nn-compare / --nn-apply: network weights file")
    ap.add_argument("--coarse-sweep", default=None, metavar="K1,K2,...",
                    help="instead of the default line: time to 1e-6 on --workload for each coarse size "
                         "(k_trial = max(8, k))")
    ap.add_argument("--nn-apply", action="store_true",
                    help="instead of the default line: time one network application to the 256 subdomains of the "
                         "1024 x 1024 workload (HIP events), with its algorithmic FLOPs")
    ap.add_argument("--nn-quick", action="store_true",
                    help="--nn-compare: only exact LU and two NN-FGMRES settings, all with one coarse function")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported "
              "(the path would shard over right-hand sides and subdomain slabs)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2509_03622_amd import nosdd
    from paper_2509_03622_amd.workloads import WORKLOADS

    if a.adjoint:
        from paper_2509_03622_amd.workloads import inverse_design_1024
        torch.cuda.init()
        w = inverse_design_1024()
        ctx = nosdd.Context(0, nosdd.torch_stream_handle())
        P = nosdd.Problem(ctx, w.eps, w.h, w.npml, w.core_x, w.core_y, w.overlap, w.wavelengths)
        t0 = time.perf_counter()
        P.setup(k_coarse=w.k_coarse, k_trial=8)
        torch.cuda.synchronize()
        setup_ms = 1e3 * (time.perf_counter() - t0)
        J = torch.from_numpy(w.J()).cuda()
        fom, grad, iters, st = P.fom_gradient(J, w.focal, max_iters=2000)      # warm-up (graphs, tuning)
        torch.cuda.synchronize()
        reps = max(1, a.steps)
        t0 = time.perf_counter()
        for _ in range(reps):
            fom, grad, iters, st = P.fom_gradient(J, w.focal, max_iters=2000)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        x0, x1, y0, y1 = w.design
        gd = grad[y0:y1, x0:x1]
        print(json.dumps({"metric": "time per inverse-design gradient (forward + adjoint solves to 1e-6)",
                          "mode": "adjoint", "n_gpus": 1, "data": "synthetic", "dtype": "c64",
                          "config": {"workload": w.name, "grid": f"{w.nx}x{w.ny}", "cores": "16x16 of 64",
                                     "wavelengths": w.wavelengths, "design_region": list(w.design),
                                     "focal": w.focal, "k_coarse": w.k_coarse},
                          "ms_per_gradient": round(ms, 1), "setup_ms": round(setup_ms, 1), "status": int(st),
                          "fom": fom, "iterations_forward": iters[0].ravel().tolist(),
                          "iterations_adjoint": iters[1].ravel().tolist(),
                          "design_grad_abs_max": float(gd.abs().max())}), flush=True)
        P.close()
        ctx.close()
        return
    if a.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy_probe", "bytes_read_per_copy": src.numel() * 4,
                          "bytes_written_per_copy": dst.numel() * 4, "copies": 3}), flush=True)
        return
    if a.paper_compare:
        torch.cuda.init()
        w = WORKLOADS[a.workload]()
        ctx = nosdd.Context(0, nosdd.torch_stream_handle())
        P = nosdd.Problem(ctx, w.eps, w.h, w.npml, w.core_x, w.core_y, w.overlap, w.wavelengths, w.pml_m,
                          w.pml_lnR, cores=w.cores)
        P.setup(k_coarse=max(w.k_coarse, 1), k_trial=w.k_trial)
        J = torch.from_numpy(w.J()).cuda()
        E = torch.zeros((len(w.wavelengths), len(w.sources), w.ny, w.nx), dtype=torch.complex64, device="cuda")
        tol = 1e-5
        rows = []
        P.solve_device(J, E, tol=tol, max_iters=3000)           # warm-up: autotuning, graphs
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist, iters, fin, st = P.solve_device(J, E, tol=tol, max_iters=3000)
        torch.cuda.synchronize()
        rows.append({"form": "FGMRES(30), two-level volume coarse correction", "status": int(st),
                     "ms": round(1e3 * (time.perf_counter() - t0), 2),
                     "iterations_per_rhs": iters.ravel().tolist(),
                     "final_rel_residual": [float(f"{v:.3e}") for v in fin.ravel()]})
        print(f"[bench] {rows[-1]}", file=sys.stderr, flush=True)
        for m, coarse in ((0.0, False), (0.3, False), (0.0, True), (0.3, True)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hist, iters, fin, st = P.solve_paper(J, E, momentum=m, coarse=coarse, tol=tol, max_iters=3000)
            torch.cuda.synchronize()
            rows.append({"form": "Algorithm 3 sweeps" + (", Robin-space coarse correction" if coarse else ""),
                         "momentum": m, "status": int(st), "ms": round(1e3 * (time.perf_counter() - t0), 2),
                         "sweeps_per_rhs": iters.ravel().tolist(),
                         "final_rel_residual": [float(f"{v:.3e}") for v in fin.ravel()]})
            print(f"[bench] {rows[-1]}", file=sys.stderr, flush=True)
        print(json.dumps({"metric": "time to 1e-5 residual per global solve: Algorithm 3 loop vs FGMRES form",
                          "mode": "paper_vs_fgmres", "n_gpus": 1, "data": "synthetic", "dtype": "c64",
                          "config": {"workload": w.name, "grid": f"{w.nx}x{w.ny}",
                                     "cores": describe_cores(w), "overlap": w.overlap,
                                     "wavelengths": w.wavelengths, "k_coarse": max(w.k_coarse, 1), "tol": tol},
                          "rows": rows}), flush=True)
        P.close()
        ctx.close()
        return
    if a.quadtree_compare:
        from paper_2509_03622_amd.workloads import quadtree_512
        torch.cuda.init()
        w = quadtree_512()
        J = torch.from_numpy(w.J()).cuda()
        rows = []
        for name, cores, cx in (("quad-tree", w.cores, None), ("uniform 8 x 8 of 64", None, [64] * 8),
                                ("uniform 16 x 16 of 32", None, [32] * 16)):
            ctx = nosdd.Context(0, nosdd.torch_stream_handle())
            P = nosdd.Problem(ctx, w.eps, w.h, w.npml, cx, cx, w.overlap, w.wavelengths, w.pml_m, w.pml_lnR,
                              cores=cores)
            t0 = time.perf_counter()
            P.setup(k_coarse=w.k_coarse, k_trial=w.k_trial)
            torch.cuda.synchronize()
            setup_ms = 1e3 * (time.perf_counter() - t0)
            E = torch.zeros((len(w.wavelengths), 1, w.ny, w.nx), dtype=torch.complex64, device="cuda")
            dt, iters, fin, st, ms_k = timed_solve(torch, P, J, E, a.max_iters, reps=max(1, a.steps))
            rows.append({"partition": name, "subdomains": P.sizes()[0], "status": int(st),
                         "time_to_tol_ms": round(1e3 * dt, 2), "setup_ms": round(setup_ms, 1),
                         "iterations_per_rhs": iters.ravel().tolist(),
                         "final_rel_residual": [float(f"{v:.3e}") for v in fin.ravel()],
                         "kernel_ms": dict(zip(("local_solve", "operator", "arnoldi", "coarse"), ms_k))})
            print(f"[bench] {rows[-1]}", file=sys.stderr, flush=True)
            P.close()
            ctx.close()
        print(json.dumps({"metric": "time to 1e-6 residual per global solve: quad-tree vs uniform partitions",
                          "mode": "quadtree_vs_uniform", "n_gpus": 1, "data": "synthetic", "dtype": "c64",
                          "config": {"workload": w.name, "grid": f"{w.nx}x{w.ny}", "overlap": w.overlap,
                                     "wavelengths": w.wavelengths, "k_coarse": w.k_coarse, "tol": 1e-6},
                          "rows": rows}), flush=True)
        return
    if a.coarse_sweep:
        torch.cuda.init()
        w = WORKLOADS[a.workload]()
        J = torch.from_numpy(w.J()).cuda()
        ctx = nosdd.Context(0, nosdd.torch_stream_handle())
        rows = []
        for kc in [int(v) for v in a.coarse_sweep.split(",")]:
            P = nosdd.Problem(ctx, w.eps, w.h, w.npml, w.core_x, w.core_y, w.overlap, w.wavelengths, w.pml_m,
                              w.pml_lnR, cores=w.cores)
            t0 = time.perf_counter()
            P.setup(k_coarse=kc, k_trial=max(8, kc))
            torch.cuda.synchronize()
            setup_ms = 1e3 * (time.perf_counter() - t0)
            E = torch.zeros((len(w.wavelengths), len(w.sources), w.ny, w.nx), dtype=torch.complex64, device="cuda")
            P.solve_device(J, E, max_iters=2)                   # autotuning and graph capture
            torch.cuda.synchronize()
            E.zero_()
            t0 = time.perf_counter()
            hist, iters, fin, st = P.solve_device(J, E, max_iters=a.max_iters)
            torch.cuda.synchronize()
            rows.append({"k_coarse": kc, "k_trial": max(8, kc), "status": int(st),
                         "time_to_tol_ms": round(1e3 * (time.perf_counter() - t0), 2),
                         "setup_ms": round(setup_ms, 1), "iterations_per_rhs": iters.ravel().tolist()})
            print(f"[bench] {rows[-1]}", file=sys.stderr, flush=True)
            P.close()
        print(json.dumps({"mode": "coarse_sweep", "metric": "time to 1e-6 residual per global solve by coarse size",
                          "config": {"workload": w.name, "grid": f"{w.nx}x{w.ny}", "wavelengths": w.wavelengths,
                                     "sources": len(w.sources)}, "rows": rows}), flush=True)
        ctx.close()
        return
    if a.nn_apply:
        torch.cuda.init()
        from paper_2509_03622_amd.workloads import blocks_1024
        w = blocks_1024()
        ctx = nosdd.Context(0, nosdd.torch_stream_handle())
        P = nosdd.Problem(ctx, w.eps, w.h, w.npml, w.core_x, w.core_y, w.overlap, w.wavelengths, w.pml_m, w.pml_lnR)
        P.setup(k_coarse=0, sub_solver=1, nn_weights=a.weights, inner_max=2, inner_tol=0.1)
        nt, lc, ne, nc = P.sizes()
        g = torch.Generator(device="cuda").manual_seed(0)
        v = torch.randn((1, lc), dtype=torch.complex64, device="cuda", generator=g)
        e = torch.empty_like(v)
        for _ in range(3):
            P.nn_apply(v, e)
        torch.cuda.synchronize()
        reps = max(a.steps, 5)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            P.nn_apply(v, e)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        tiles = tile_geometry(w)
        C, m, L, hid = 64, 16, 4, 128

        def parts(lx, ly):
            """Algorithmic FLOPs of one network application to one lx x ly subdomain:
            (channel contractions on BF16 MFMA, truncated DFTs, DFT products executed on BF16
            MFMA with high/low operand splits, other FP32 work)."""
            n = lx * ly
            fy, fx = 64 * lx * m * ly * 4, 64 * m * 2 * m * lx * 8          # forward y (real input), then x
            ix, iy = 64 * m * lx * 2 * m * 8, 64 * lx * ly * m * 4          # inverse x, then y (real output)
            mix = 2 * m * m * C * C * 8
            bf16 = L * (mix + 2 * C * C * n) + 2 * C * hid * n
            dft = L * (fy + fx + ix + iy)
            dft_exec = L * (2 * fy + 3 * fx + 3 * ix + 3 * iy)             # products per k step: 2, 3, 3, 3
            other = 2 * 9 * C * n + 2 * hid * 2 * n                        # lift, last projection layer
            return bf16, dft, dft_exec, other
        tot = [sum(parts(t[0], t[1])[i] for t in tiles) for i in range(4)]
        bf16_part, dft_part, dft_exec, other = tot
        total = bf16_part + dft_part + other
        floor_us = 1e6 * ((bf16_part + dft_exec) / 2.5e15 + other / FP32_MFMA_PEAK_TFS / 1e12)
        print(json.dumps({"mode": "nn_apply", "metric": "one network application to every subdomain",
                          "config": {"workload": w.name, "subdomains": nt, "weights": os.path.basename(a.weights)},
                          "ms_per_application": round(ms, 4), "reps": reps,
                          "algorithmic_gflop": round(total / 1e9, 2),
                          "bf16_mfma_gflop": round(bf16_part / 1e9, 2), "dft_gflop": round(dft_part / 1e9, 2),
                          "dft_bf16_executed_gflop": round(dft_exec / 1e9, 2), "fp32_other_gflop": round(other / 1e9, 2),
                          "achieved_tflops": round(total / (ms * 1e-3) / 1e12, 2),
                          "mfma_floor_us": round(floor_us, 1)}), flush=True)
        P.close()
        ctx.close()
        return
    if a.nn_compare:
        torch.cuda.init()
        if a.nn_quick:
            configs = [(1, "lu", 0, 0.0), (1, "nn", 2, 0.1), (1, "nn", 4, 0.01)]
        else:
            configs = [(kc, "lu", 0, 0.0) for kc in (0, 1)]
            configs += [(kc, "nn", n, t) for kc in (1, 0) for n, t in ((1, 0.1), (2, 0.1), (4, 0.1), (4, 0.01),
                                                                     (8, 0.01))]
        w, rows = nn_compare(torch, nosdd, "blocks1024", configs, max_iters=3000, weights=a.weights)
        lu = min((r for r in rows if r["solver"] == "lu" and r["status"] == 0), key=lambda r: r["time_to_tol_ms"])
        nn = [r for r in rows if r["solver"] == "nn" and r["status"] == 0]
        best = min(nn, key=lambda r: r["time_to_tol_ms"]) if nn else None
        print(json.dumps({"metric": METRIC, "mode": "nn_vs_lu", "n_gpus": 1, "data": "synthetic",
                          "config": {"workload": w.name, "grid": f"{w.nx}x{w.ny}", "cores": "16x16 of 64",
                                     "overlap": w.overlap, "wavelengths": w.wavelengths, "tol": 1e-6,
                                     "network": "FNO C=64, 16 modes, 4 layers, BF16 MFMA, FP32 accumulation",
                                     "weights": os.path.basename(a.weights)},
                          "best_lu_ms": lu["time_to_tol_ms"],
                          "best_nn_ms": best["time_to_tol_ms"] if best else None,
                          "nn_over_lu_time": round(best["time_to_tol_ms"] / lu["time_to_tol_ms"], 3) if best else None,
                          "rows": rows}), flush=True)
        return

    w = WORKLOADS[a.workload]()
    n_wl, n_src = len(w.wavelengths), len(w.sources)
    n_rhs = n_wl * n_src
    tiles = tile_geometry(w)
    multi = n_src >= 4 and max(min(t[0], t[1]) for t in tiles) <= 112
    # algorithmic work of the dominant kernel, per (subdomain, RHS) solve
    flops_per_unit = float(np.mean([8 * min(t[0], t[1]) ** 2 * (2 * max(t[0], t[1]) - 1) for t in tiles]))
    if multi:
        # many-source kernel: each factor stream is shared by a group of sources
        # (32 for blocks up to 80 cells, 16 above)
        def groups(t):
            return -(-n_src // (32 if min(t[0], t[1]) <= 80 else 16))
        stream = float(np.mean([groups(t) * 8 * (2 * max(t[0], t[1]) - 1) * min(t[0], t[1])
                                * (min(t[0], t[1]) + 2) // 2 for t in tiles]))
        io = float(np.mean([8 * (t[0] * t[1] + t[2]) for t in tiles]))
        bytes_per_unit = io + stream / n_src          # per (subdomain, RHS)
    else:
        bytes_per_unit = float(np.mean([local_solve_bytes(*t) for t in tiles]))
    restart = a.restart

    torch.cuda.init()
    dev = torch.device("cuda:0")
    ctx = nosdd.Context(0, nosdd.torch_stream_handle())
    P = nosdd.Problem(ctx, w.eps, w.h, w.npml, w.core_x, w.core_y, w.overlap, w.wavelengths, w.pml_m, w.pml_lnR,
                      cores=w.cores)
    t0 = time.perf_counter()
    P.setup(k_coarse=w.k_coarse, k_trial=w.k_trial)
    torch.cuda.synchronize()
    setup_ms = 1e3 * (time.perf_counter() - t0)
    J = torch.from_numpy(w.J()).to(dev)
    E = torch.zeros((n_wl, n_src, w.ny, w.nx), dtype=torch.complex64, device=dev)

    # 1. time to tol: one complete solve of every RHS to 1e-6 (autotuning and
    #    graph capture happen in a first, short call)
    P.solve_device(J, E, tol=1e-6, max_iters=2)
    torch.cuda.synchronize()
    E.zero_()
    if a.no_full_solve:
        time_to_tol, iters_full, fin_full, st_full = float("nan"), np.zeros(1, int), np.zeros(1), -1
    else:
        t0 = time.perf_counter()
        hist, iters_full, fin_full, st_full = P.solve_device(J, E, tol=1e-6, max_iters=a.max_iters)
        torch.cuda.synchronize()
        time_to_tol = time.perf_counter() - t0
        print(f"[bench] full solve: {time_to_tol:.2f} s, status {st_full}, iterations per RHS "
              f"{iters_full.ravel().tolist()}", file=sys.stderr, flush=True)

    # 2. steps: one FGMRES(restart) cycle over every RHS per step, each
    #    continuing from the previous step's field
    X = torch.zeros_like(E)

    def cycle():
        return P.solve_device(J, X, tol=1e-6, restart=restart, max_iters=restart, x0=X)
    for _ in range(a.warmup):
        cycle()
    torch.cuda.synchronize()
    tot_units = 0
    live_iters = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        hist, iters, fin, st = cycle()
        tot_units += int(iters.sum()) * len(tiles)
        live_iters.append(iters)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    steps_full = all(int(v) == restart for it in live_iters for v in it.ravel())
    print(f"[bench] timed {a.steps} cycles in {elapsed:.3f} s (every RHS active in every step: {steps_full})",
          file=sys.stderr, flush=True)
    # kernel classes: one more cycle, launched kernel by kernel with HIP events
    # on the library stream around every launch group
    P.profile(True)
    cycle()
    torch.cuda.synchronize()
    P.profile(False)
    ms_k, launches, units = P.kernel_times()

    ms_per_step = 1e3 * elapsed / max(a.steps, 1)
    value = tot_units / elapsed
    lu_ms = ms_k[0]
    per_launch_units = units[0] / max(launches[0], 1)
    lu_bytes = units[0] * bytes_per_unit
    lu_flops = units[0] * flops_per_unit
    achieved_gbs = lu_bytes / (lu_ms * 1e-3) / 1e9 if lu_ms > 0 else 0.0
    achieved_tf = lu_flops / (lu_ms * 1e-3) / 1e12 if lu_ms > 0 else 0.0
    kname = ("bt_solve_multi_kernel (gather + block-Thomas subdomain LU for a group of sources sharing each factor "
             "block, FP32 MFMA products, core scatter)" if multi else
             "bt_solve_kernel (gather + block-Thomas subdomain LU solve + core scatter)")
    if multi and achieved_tf / FP32_MFMA_PEAK_TFS >= achieved_gbs / HBM_PEAK_GBS:
        roofline = {"bound": "mfma", "achieved": round(achieved_tf, 2), "peak": FP32_MFMA_PEAK_TFS,
                    "unit": "TFLOP/s", "frac": round(achieved_tf / FP32_MFMA_PEAK_TFS, 4)}
    else:
        roofline = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved_gbs / HBM_PEAK_GBS, 4)}
    roofline.update({"traffic": read_traffic(per_launch_units, multi), "kernel": kname,
                     "avg_launch_us": round(1e3 * lu_ms / max(launches[0], 1), 2),
                     "algorithmic_flops_per_launch": round(per_launch_units * flops_per_unit),
                     "algorithmic_bytes_per_launch": round(per_launch_units * bytes_per_unit),
                     "hbm_frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
                     "fp32_mfma_frac": round(achieved_tf / FP32_MFMA_PEAK_TFS, 4),
                     "launches": int(launches[0])})
    share = {k: round(float(v), 3) for k, v in zip(("local_solve", "operator", "arnoldi", "coarse"), ms_k)}
    out = {"metric": METRIC, "value": round(value, 1), "unit": "subdomain solves/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_per_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
           "data": "synthetic",
           "config": {"workload": w.name, "grid": f"{w.nx}x{w.ny}", "cores": describe_cores(w),
                      "overlap": w.overlap, "wavelengths": w.wavelengths, "sources": n_src, "rhs": n_rhs,
                      "k_coarse": w.k_coarse, "subdomain_solver": "exact LU (block-Thomas)",
                      "restart": restart, "tol": 1e-6,
                      "step": f"one FGMRES({restart}) restart cycle of all {n_rhs} right-hand sides: {restart} "
                              "two-level Schwarz sweeps (gather, subdomain solves, scatter, operator, coarse "
                              "correction) with their Arnoldi steps, the cycle's explicit FP64 residual and update"},
           "time_to_tol_ms": None if a.no_full_solve else round(1e3 * time_to_tol, 1),
           "time_to_tol_status": int(st_full),
           "outer_iterations_per_rhs": iters_full.ravel().tolist(),
           "final_rel_residual": [float(f"{v:.3e}") for v in fin_full.ravel()],
           "every_rhs_active_in_timed_steps": steps_full,
           "setup_ms": round(setup_ms, 1),
           "kernel_ms_per_step": share,
           "launch_parameters": P.tuning(),
           "roofline": roofline}

    if not a.no_stencil:
        P.close()
        out["stencil_roofline"] = stencil_roofline(torch, nosdd)
        print(f"[bench] stencil roofline {out['stencil_roofline']}", file=sys.stderr, flush=True)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_iters, direct=not a.no_direct)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
