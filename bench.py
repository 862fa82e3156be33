"""Benchmark of the VCT-SPH(2) operator path on one MI355X.

One step = one pass of the whole hot path over the 3-D sigma-SPH particle set
(512 x 512 x 32 = 8,388,608 particles, sloped-beach bathymetry, 5% jitter):
  cell sort -> neighbour lists (one staged search) -> FP64 moments + solve (the
  FP32 state only) -> mixed-precision operator apply (grad + lap + cross) ->
  FP64 state of the adjoint's rows, solved again from the moment sums the
  forward kept -> FP64 apply of those rows -> adjoint (d/dphi and d/d
  bathymetry coefficients).  --adjoint-state recompute runs both moment sweeps
  again in the backward instead.
Inputs are resident in HBM before the timed region.  `value` is particle-
operator evaluations (particles x fields) per second of the whole step.

The JSON line also carries per-stage times, per-kernel launch times (HIP
events on the launch stream, recorded by the library over the timed steps),
the apply-only rates of the FP64 and mixed paths, the roofline of the step's
dominant kernel and of the mixed apply kernel (algorithmic bytes or flops per
launch / average launch time), and the CPU oracle timed on a bounded sample of
the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6

# Algorithmic floating-point operations (a fused multiply-add counts 2, a
# square root or reciprocal 1) of the 3-D kernels, counted from the per-pair
# arithmetic they perform:
#   moment sweeps, per pair: pass 1 = offsets and q^2 (11), the 6 pair and 10
#   cubic monomials (16), kernel value times volume (8), A and B sums (32);
#   pass 2 = offsets and q^2 (11), monomials (16), r~.L~.r~ (12), weight (12),
#   C sums (20), E sums of the 15 quartic monomials (45);
#   moment solve, per particle: the Schur LU and folds (about 3200);
#   adjoint d/dphi (push form), per directed neighbour entry: the method needs one
#   Laplacian weight W_ik per entry (the row sums u_k sum_j W_kj are a
#   by-product of the same weights): offsets and q^2 (11), pair monomials (6),
#   kernel value and 1/q^4 (10), r~.L~.r~ (12), the Laplacian row contraction
#   (18), the combination and the sum (5);
#   neighbour search, per candidate: offset difference, squared distance and
#   the two comparisons in FP32 (9).
MOMENT_FLOP_PER_PAIR_3D = (11 + 16 + 8 + 32) + (11 + 16 + 12 + 12 + 20 + 45)
MOMENT_FLOP_SOLVE_3D = 3200
ADJOINT_DPHI_FLOP_PER_ENTRY_3D = 11 + 6 + 10 + 12 + 18 + 5
NB_FLOP_PER_CANDIDATE = 9
FP32_VALU_PEAK_TFLOPS = 157.3        # published FP32 vector peak (packed instructions)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--config", default="c3")
    p.add_argument("--nf", type=int, default=1)
    p.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--adjoint-state", choices=["forward", "resolve", "recompute"], default="forward",
                   help="backward state: folded by the forward's solve beside its own, solved again from the "
                        "forward's kept moment sums, or sweeps + solve again")
    p.add_argument("--no-grad-hint", action="store_true",
                   help="the backward's FP64 apply computes its own first-pass gradient instead of reading the "
                        "forward's")
    p.add_argument("--ppe-iters", type=int, default=100, help="BiCGSTAB iterations of the pressure-step measurement")
    p.add_argument("--skip", default="",
                   help="comma-separated side measurements to leave out (outside the timed steps): "
                        "fd (adjoint central difference), ppe, jbar, r2 -- for profiler runs")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a 1 GiB device-to-device copy five times (reference for HBM byte counters)")
    return p.parse_args()


def kernel_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_2607_28872_amd", "csrc"))):
        h.update(open(os.path.join(ROOT, "paper_2607_28872_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def progress(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def measured_traffic(kernel_name, launches_bytes):
    """HBM bytes per launch from committed rocprofv3 counter summaries, or None
    if absent or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_hash():
        return None
    k = d.get("kernels", {}).get(kernel_name)
    if not k:
        return None
    return (k["fetch_kib"] * d["fetch_scale"] + k["write_kib"] * d["write_scale"]) * 1024.0


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (asked for {args.gpus}); "
              "sharding across GPUs is designed (spatial slabs with halo exchanges) but not implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8, "copies": 5}))
        return

    from paper_2607_28872_amd import inputs as I
    from paper_2607_28872_amd import vct

    dev = "cuda:0"
    torch.cuda.set_device(0)
    w = I.config(args.config)
    progress(f"workload {args.config}: {w.n} particles generated")
    n, dim = w.n, w.dim
    nf = args.nf
    phis = np.concatenate([w.phi] * ((nf + w.phi.shape[0] - 1) // w.phi.shape[0]))[:nf]
    theta = I.theta0()
    ms = w.mapspec.with_terms(I.theta_terms(theta))
    cmap = vct.make_map(ms)
    target = I.target_field(w.pos, ms.Hhat)
    L = vct.lib()

    # ---------------------------------------------------------------- resident inputs + buffers
    pos = torch.as_tensor(w.pos, device=dev).contiguous()
    # the per-particle input fields in one (2 + nf, n) array: volume, the
    # fields, the loss target; one gather brings them all into sorted order
    fields_in = torch.as_tensor(np.concatenate([w.vol[None], phis, target[None]]), device=dev).contiguous()
    ncell, _ = vct.vct_grid_dims(dim, w.lo, w.hi, w.R)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    pos_s = torch.empty((dim, n), dtype=torch.float64, device=dev)
    fields_s = torch.empty((2 + nf, n), dtype=torch.float64, device=dev)
    vol_s, phi_s, g_s = fields_s[0], fields_s[1:1 + nf], fields_s[1 + nf]
    cell_start = torch.empty(ncell + 1, dtype=torch.int64, device=dev)
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    _, dims = vct.vct_grid_dims(dim, w.lo, w.hi, w.R)
    ncols = dims[0] * dims[1] if dim == 3 else dims[0]
    cap = L.vct_chunk_capacity(dim, n, ncell)
    chunk_off = torch.empty(ncols + 1, dtype=torch.int64, device=dev)
    chunk_start = torch.empty(cap + 1, dtype=torch.int32, device=dev)
    chunk_info = torch.empty((cap, 4), dtype=torch.int32, device=dev)
    chunk_win = torch.empty((cap, 32), dtype=torch.int32, device=dev)
    ws_cells = torch.empty(L.vct_build_cells_workspace_size(dim, n, ncell), dtype=torch.uint8, device=dev)
    ws_nb = torch.empty(L.vct_neighbors_workspace_size(n, ncell), dtype=torch.uint8, device=dev)
    ws_mom = torch.empty(L.vct_moments_workspace_size(dim, n), dtype=torch.uint8, device=dev)
    nterms = cmap.nterms

    fwd_mask = vct.VCT_OUT_DEFAULT
    # the adjoint's rows: the Laplacian (for u) and the projected derivatives
    # whose mapping coefficients depend on the bathymetry (for dtheta)
    adj_mask = vct.VCT_OUT_LAP | vct.VCT_OUT_PZ
    n_out = vct.vct_n_out(dim, fwd_mask)
    stride_f = vct.vct_state_stride(dim, fwd_mask)
    stride_a = vct.vct_state_stride(dim, adj_mask)
    st64 = torch.empty((stride_f, n), dtype=torch.float64, device=dev)
    st32 = torch.empty((stride_f, n), dtype=torch.float32, device=dev)
    sta = torch.empty((stride_a, n), dtype=torch.float64, device=dev)
    flags = torch.empty(n, dtype=torch.uint8, device=dev)
    out = torch.empty((nf, n, n_out), dtype=torch.float64, device=dev)
    proj = torch.empty((1, n, vct.vct_n_out(dim, adj_mask)), dtype=torch.float64, device=dev)
    # the forward's first-pass gradient of each field, read back by the
    # backward's FP64 apply of field 0 (same field, geometry and neighbours)
    ghint = None if args.no_grad_hint else torch.empty((nf, dim, n), dtype=torch.float32, device=dev)
    u = torch.empty(n, dtype=torch.float64, device=dev)
    dphi = torch.empty(n, dtype=torch.float64, device=dev)
    dth = torch.empty(nterms, dtype=torch.float64, device=dev)

    # size the column array once (the geometry does not change between steps)
    vct.vct_build_cells(dim, n, pos, w.lo, w.hi, w.R, perm, pos_s, cell_start, ncell, ws_cells)
    nl0 = vct.make_nlist(dim, n, ncell, w.lo, w.hi, w.R, cell_start, chunk_off, chunk_start, chunk_info, row_ptr)
    _, nnz = vct.vct_neighbors(nl0, pos_s, 0, 0, ws_nb)
    col16 = torch.empty(max(nnz, 8), dtype=torch.uint16, device=dev)
    # the adjoint takes its push form (no int32 columns, no transposed-entry
    # map): the geometry is rebuilt every step, and building the map costs more
    # than it saves in a single adjoint call
    nl = vct.make_nlist(dim, n, ncell, w.lo, w.hi, w.R, cell_start, chunk_off, chunk_start, chunk_info, row_ptr,
                        None, col16, chunk_win=chunk_win)
    ws_adj = torch.empty(L.vct_adjoint_workspace_size(dim, n, nnz, nterms), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    stage_names = ["cells", "nb", "moments", "apply", "moments_adj", "adjoint"]
    # the sorted copies of the volumes and fields are gathered on a second
    # stream (default priority) while the neighbour search, which reads only
    # the sorted positions, runs on the first
    side = torch.cuda.Stream(device=dev)
    ev_perm, ev_fields = torch.cuda.Event(), torch.cuda.Event()

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    def step(record):
        marks = [ev()] if record else None

        def mark():
            if record:
                marks.append(ev())

        vct.vct_build_cells(dim, n, pos, w.lo, w.hi, w.R, perm, pos_s, cell_start, ncell, ws_cells)
        ev_perm.record(stream)
        side.wait_event(ev_perm)
        vct.vct_gather_sorted(n, 2 + nf, perm, fields_in, fields_s, stream=side)
        ev_fields.record(side)
        mark()
        vct.vct_neighbors(nl, pos_s, nnz, 0, ws_nb)
        stream.wait_event(ev_fields)
        mark()
        # the forward only runs the mixed apply: the FP32 state is all it reads
        # (its solve also folds the backward's FP64 rows from the same inverse)
        if args.adjoint_state == "forward":
            vct.vct_moments_ex(nl, pos_s, vol_s, w.kernel, cmap, fwd_mask, None, st32, adj_mask, sta, None, flags,
                               False, ws_mom)
        else:
            vct.vct_moments(nl, pos_s, vol_s, w.kernel, cmap, fwd_mask, None, st32, flags, False, ws_mom)
        mark()
        vct.vct_apply_ops_ex(nl, nf, phi_s, pos_s, vol_s, w.kernel, st32, fwd_mask, vct.VCT_MIXED, out, g_out=ghint)
        mark()
        # backward of loss = sum (lap f - g)^2: the FP64 state of its rows,
        # from the moment sums the forward left in ws_mom (or recomputed)
        if args.adjoint_state == "resolve":
            vct.vct_moments_resolve(nl, pos_s, cmap, adj_mask, sta, None, flags, False, ws_mom)
        elif args.adjoint_state == "recompute":
            vct.vct_moments(nl, pos_s, vol_s, w.kernel, cmap, adj_mask, sta, None, flags, False, ws_mom)
        mark()
        vct.vct_apply_ops_ex(nl, 1, phi_s, pos_s, vol_s, w.kernel, sta, adj_mask, vct.VCT_FP64, proj,
                             g_in=None if ghint is None else ghint[0])
        torch.sub(proj[0, :, 0], g_s, out=u)
        u.mul_(2.0)
        vct.vct_apply_ops_adjoint(nl, pos_s, vol_s, w.kernel, sta, adj_mask, cmap, proj, u, dphi, dth, ws_adj)
        mark()
        return marks

    progress(f"buffers ready, {nnz} neighbour entries; warm-up")
    for _ in range(args.warmup):
        step(False)
    # one more untimed step with launch timing on, so that the events the
    # timed steps record are already created
    vct.vct_timing_enable(True)
    step(False)
    torch.cuda.synchronize()
    vct.vct_timing_enable(False)
    vct.vct_timing_reset()
    stage_ms = {k: [] for k in stage_names}
    progress(f"timing {args.steps} steps")
    vct.vct_timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        marks = step(True)
        torch.cuda.synchronize()
        for k, nm in enumerate(stage_names):
            stage_ms[nm].append(marks[k].elapsed_time(marks[k + 1]))
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps
    vct.vct_timing_enable(False)
    ktimes = vct.vct_timing_read()
    stage = {k: float(np.mean(v)) for k, v in stage_ms.items()}

    # apply-only rates of both precisions (same launch configuration)
    def time_apply(prec, state, reps=10):
        vct.vct_apply_ops(nl, nf, phi_s, pos_s, vol_s, w.kernel, state, fwd_mask, prec, out)
        torch.cuda.synchronize()
        e0 = ev()
        for _ in range(reps):
            vct.vct_apply_ops(nl, nf, phi_s, pos_s, vol_s, w.kernel, state, fwd_mask, prec, out)
        e1 = ev()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    vct.vct_moments(nl, pos_s, vol_s, w.kernel, cmap, fwd_mask, st64, st32, flags, False, ws_mom)
    progress("apply-only timing")
    t_apply_mixed = time_apply(vct.VCT_MIXED, st32)
    t_apply_fp64 = time_apply(vct.VCT_FP64, st64)

    deg = nnz / n
    # algorithmic bytes of one apply launch: row_ptr, 16-bit columns, one read
    # of every particle's position/volume/field, the state, the outputs
    def apply_bytes(state_elem):
        per_particle = 8 + 2 * deg + (dim * 8 + 8 + 8 * nf) + stride_f * state_elem + 8 * n_out * nf
        return per_particle * n

    b_mixed, b_fp64 = apply_bytes(4), apply_bytes(8)
    # the step's forward also writes the first-pass gradient (FP32, d per
    # field) that the backward's FP64 apply reads instead of its first pass
    b_hint = 0 if args.no_grad_hint else 4 * dim * n
    b_mixed_step = b_mixed + b_hint * nf
    # per-kernel launch times over the timed steps, and the roofline of the
    # kernel that takes the most time per step
    n_out_a = vct.vct_n_out(dim, adj_mask)
    pairs = float(nnz)
    b_fp64_adj = n * (8 + 2 * deg + (dim * 8 + 8 + 8) + stride_a * 8 + 8 * n_out_a)
    candidates = n * 27.0 * (n / ncell)
    models = {   # kernel -> (bound, algorithmic bytes or flops per launch, peak)
        "k_apply (mixed)": ("hbm", b_mixed_step, HBM_PEAK_GBS),
        "k_apply (fp64)": ("hbm", b_fp64_adj, HBM_PEAK_GBS),
        "k_apply (fp64, given G)": ("hbm", b_fp64_adj + b_hint, HBM_PEAK_GBS),
        "k_moment_sweeps": ("alu", pairs * MOMENT_FLOP_PER_PAIR_3D, FP64_PEAK_TFLOPS),
        "k_moment_solve": ("alu", n * MOMENT_FLOP_SOLVE_3D, FP64_PEAK_TFLOPS),
        "k_adjoint_push": ("alu", pairs * ADJOINT_DPHI_FLOP_PER_ENTRY_3D, FP64_PEAK_TFLOPS),
        "k_nb_chunk (stage)": ("alu", candidates * NB_FLOP_PER_CANDIDATE, FP32_VALU_PEAK_TFLOPS),
    }
    kernels = {k: {"launches_per_step": c / args.steps, "ms_per_step": round(t / args.steps, 4),
                   "avg_launch_ms": round(t / c, 4)} for k, (c, t) in sorted(ktimes.items())}

    def kernel_roofline(name):
        c, t = ktimes[name]
        avg = t / c
        bound, work, peak = models[name]
        if bound == "hbm":
            ach = work / (avg * 1e-3) / 1e9
            unit = "GB/s"
        else:
            ach = work / (avg * 1e-3) / 1e12
            unit = "TFLOP/s"
        return {"kernel": name, "bound": bound, "achieved": round(ach, 3), "peak": peak, "unit": unit,
                "frac": round(ach / peak, 4), "traffic": measured_traffic(name, work), "avg_launch_ms": round(avg, 4),
                "launches_per_step": c / args.steps, "work_per_launch": work}

    dom = max(ktimes, key=lambda k: ktimes[k][1])
    roofline = kernel_roofline(dom) if dom in models else {"kernel": dom, "bound": None, "traffic": None}
    roof_apply = kernel_roofline("k_apply (mixed)")
    roof_apply["apply_only_ms"] = round(t_apply_mixed, 4)

    # measured device-copy bandwidth (1 GiB read + 1 GiB written), the
    # attainable HBM figure beside the vendor peak
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = ev()
    for _ in range(5):
        dst.copy_(src)
    e1 = ev()
    torch.cuda.synchronize()
    copy_gbs = 2.0 * src.numel() * 8 * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    for r in (roofline, roof_apply):
        if r.get("bound") == "hbm":
            r["frac_of_copy"] = round(r["achieved"] / copy_gbs, 4)

    value = n * nf / t_step
    res = {
        "metric": "particle-operator evals/s (grad+lap+cross), mixed vs FP64 GPU; HBM GB/s",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-sums/f64-moments",
        "data": "synthetic",
        "config": {"workload": f"3-D sigma-SPH sloped beach {w.counts[0]}x{w.counts[1]}x{w.counts[2]} "
                               f"({n} particles), Wendland C2 R=3dx, 5% jitter, {nf} field(s), mixed apply, "
                               + {"forward": "adjoint state folded by the forward's solve",
                                  "resolve": "adjoint state solved from the forward's moment sums",
                                  "recompute": "adjoint with recomputed moments"}[args.adjoint_state]
                               + ("" if args.no_grad_hint else ", backward reads the forward's first-pass gradient"),
                   "particles": n, "fields": nf, "neighbours_per_particle": round(deg, 2),
                   "parallelism": "single GPU"},
        "stage_ms": {k: round(v, 4) for k, v in stage.items()},
        "apply_only": {"mixed_ms": round(t_apply_mixed, 4), "fp64_ms": round(t_apply_fp64, 4),
                       "mixed_evals_per_s": n * nf / (t_apply_mixed * 1e-3),
                       "fp64_evals_per_s": n * nf / (t_apply_fp64 * 1e-3),
                       "speedup_mixed_vs_fp64": round(t_apply_fp64 / t_apply_mixed, 3),
                       "fp64_alg_GBs": round(b_fp64 / (t_apply_fp64 * 1e-3) / 1e9, 1)},
        "roofline": roofline,
        "roofline_apply": roof_apply,
        "copy_GBs": round(copy_gbs, 1),
        "kernels": kernels,
    }

    # side measurements, outside the timed steps
    skip = set(x for x in args.skip.split(",") if x)
    if "fd" not in skip:
        res["adjoint_fd"] = adjoint_fd_check(vct, nl, w, phi_s, pos_s, vol_s, sta, adj_mask, proj, g_s, dphi, n, dev)
    if "ppe" not in skip:
        res["ppe"] = ppe_measure(args, w, vct, L, nl, pos_s, vol_s, sta, adj_mask, ms, perm, dev)
    if "jbar" not in skip:
        res["jbar"] = jbar_measure(w, vct, L, nl, pos_s, cmap, perm, dev)
    if "r2" not in skip:
        res["adjoint_r2"] = r2_measure(w, vct, L, nl, dim, n, pos_s, vol_s, phi_s, g_s, cmap, dev)

    if not args.no_cpu_baseline:
        progress("CPU oracle on a sample")
        cb, rows, rec = cpu_baseline(w, phis, ms, args.cpu_seconds)
        res["cpu_baseline"] = cb
        # per-operator errors of both GPU paths against the oracle at the sampled particles
        inv = np.empty(n, dtype=np.int64)
        inv[perm.cpu().numpy().astype(np.int64)] = np.arange(n)
        idx = torch.as_tensor(inv[rows], device=dev)
        vct.vct_moments(nl, pos_s, vol_s, w.kernel, cmap, fwd_mask, st64, st32, flags, False, ws_mom)
        errs = {"sample": int(len(rows)), "bars": {"grad": 1e-5, "lap_cross": 1e-4, "fp64": 1e-12}}
        for prec, state, nm in ((vct.VCT_FP64, st64, "fp64"), (vct.VCT_MIXED, st32, "mixed")):
            vct.vct_apply_ops(nl, nf, phi_s, pos_s, vol_s, w.kernel, state, fwd_mask, prec, out)
            errs[nm] = operator_errors(out[:, idx, :].cpu().numpy(), rec, dim)
        res["error_vs_oracle"] = errs
    print(json.dumps(res), flush=True)


def adjoint_fd_check(vct, nl, w, phi_s, pos_s, vol_s, sta, adj_mask, proj, g_s, dphi, n, dev):
    """The adjoint's d loss / d phi along a seeded direction v against the
    central difference of the loss with the FP64 Laplacian.  The loss is
    quadratic in phi and the difference of squares is formed as
    (a - b)(a + b - 2 g), so the central difference is exact up to rounding."""
    import torch
    progress("adjoint against a central difference")
    fd_step = 1e-6
    v = torch.randn(n, generator=torch.Generator().manual_seed(17), dtype=torch.float64).to(dev)
    lap_pm = []
    for sgn in (1.0, -1.0):
        ph = (phi_s[0] + sgn * fd_step * v).unsqueeze(0).contiguous()
        o = torch.empty_like(proj)
        vct.vct_apply_ops(nl, 1, ph, pos_s, vol_s, w.kernel, sta, adj_mask, vct.VCT_FP64, o)
        lap_pm.append(o[0, :, 0])
    a, b = lap_pm
    fd = float(((a - b) * (a + b - 2.0 * g_s)).sum().item()) / (2.0 * fd_step)
    adj = float(torch.dot(dphi, v).item())
    return {"quantity": "d loss / d phi along a seeded normal direction, loss = sum (lap f - g)^2",
            "step": fd_step, "central_difference": fd, "adjoint": adj, "rel_err": abs(fd - adj) / abs(adj)}


def ppe_measure(args, w, vct, L, nl, pos_s, vol_s, sta, mask, ms, perm, dev):
    """The pressure step on the benchmark geometry (outside the timed
    steps): the right-hand side of Eq. VCT_ppe from a smooth test velocity,
    Dirichlet rows on the boundary layer of width R, then a fixed budget of
    BiCGSTAB iterations with the FP64 Laplacian (the adjoint's state, which
    holds the LAP row) as the matrix-free operator."""
    import numpy as np
    import torch
    from paper_2607_28872_amd import inputs as I
    progress("pressure step")
    n, dim = w.n, w.dim
    cmap = vct.make_map(ms)
    idx = perm[:n].long().cpu().numpy()
    dirichlet = torch.as_tensor(I.boundary_layer(w.pos, w.lo, w.hi, w.R).astype(np.uint8)[idx], device=dev)
    v = torch.as_tensor(np.ascontiguousarray(I.velocity_field(w.pos)[:, idx]), device=dev)
    rhs = torch.empty(n, dtype=torch.float64, device=dev)
    ws = torch.empty(L.vct_ppe_workspace_size(dim, n, mask), dtype=torch.uint8, device=dev)
    p = torch.zeros(n, dtype=torch.float64, device=dev)
    vct.vct_ppe_rhs(nl, pos_s, vol_s, w.kernel, sta, mask, cmap, v, 1.0, 1e-3, 0.1, None, dirichlet, None, rhs)
    vct.vct_ppe_solve(nl, pos_s, vol_s, w.kernel, sta, mask, dirichlet, rhs, p, 1e-30, 8, ws)   # warm-up
    iters = args.ppe_iters
    p.zero_()
    vct.vct_timing_reset()
    vct.vct_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vct.vct_ppe_rhs(nl, pos_s, vol_s, w.kernel, sta, mask, cmap, v, 1.0, 1e-3, 0.1, None, dirichlet, None, rhs)
    st, it, rr = vct.vct_ppe_solve(nl, pos_s, vol_s, w.kernel, sta, mask, dirichlet, rhs, p, 1e-30, iters, ws)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    vct.vct_timing_enable(False)
    kt = vct.vct_timing_read()
    vct.vct_timing_reset()
    matvec = kt.get("k_apply (fp64)", (0, 0.0))
    return {"what": "pressure Poisson solve (Eq. VCT_ppe): BiCGSTAB, Jacobi preconditioner, SPH(2) Laplacian "
                    "matrix-free; fixed iteration budget (tol 0), rhs from a smooth velocity, Dirichlet boundary layer",
            "iterations": it, "relres": rr, "ms_total": round(t * 1e3, 3),
            "ms_per_iteration": round(t * 1e3 / max(it, 1), 4),
            "matvec_avg_ms": round(matvec[1] / max(matvec[0], 1), 4), "matvecs": matvec[0],
            "kernels": {k: {"launches": c, "avg_ms": round(ms_ / c, 4)} for k, (c, ms_) in sorted(kt.items())}}


def r2_measure(w, vct, L, nl2, dim, n, pos_s, vol_s, phi_s, g_s, cmap, dev, reps=3):
    """The bathymetry adjoint with physical positions fixed (reading R2) on
    the benchmark geometry (outside the timed steps): the FP64 state and apply
    of LAP + PGRAD + PHESS first (untimed), then the timed adjoint calls."""
    import torch
    progress("R2 adjoint")
    mask = vct.VCT_OUT_LAP | vct.VCT_OUT_PGRAD | vct.VCT_OUT_PHESS
    stride = vct.vct_state_stride(dim, mask)
    st = torch.empty((stride, n), dtype=torch.float64, device=dev)
    flags = torch.empty(n, dtype=torch.uint8, device=dev)
    ws_mom = torch.empty(L.vct_moments_workspace_size(dim, n), dtype=torch.uint8, device=dev)
    vct.vct_moments(nl2, pos_s, vol_s, w.kernel, cmap, mask, st, None, flags, False, ws_mom)
    del ws_mom
    proj = torch.empty((1, n, vct.vct_n_out(dim, mask)), dtype=torch.float64, device=dev)
    vct.vct_apply_ops(nl2, 1, phi_s[:1].contiguous(), pos_s, vol_s, w.kernel, st, mask, vct.VCT_FP64, proj)
    u = (2.0 * (proj[0, :, 0] - g_s)).contiguous()
    phi0 = phi_s[0].contiguous()
    nt = cmap.nterms
    dth = torch.empty(max(nt, 1), dtype=torch.float64, device=dev)
    ws = torch.empty(L.vct_adjoint_r2_workspace_size(dim, n, nt), dtype=torch.uint8, device=dev)
    vct.vct_apply_ops_adjoint_r2(nl2, pos_s, vol_s, w.kernel, st, mask, cmap, proj, phi0, u, dth, None, ws)
    torch.cuda.synchronize()
    vct.vct_timing_reset()
    vct.vct_timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        vct.vct_apply_ops_adjoint_r2(nl2, pos_s, vol_s, w.kernel, st, mask, cmap, proj, phi0, u, dth, None, ws)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    vct.vct_timing_enable(False)
    kt = vct.vct_timing_read()
    vct.vct_timing_reset()
    return {"what": "d loss / d bathymetry coefficients with physical positions fixed (reading R2): per-row "
                    "first sweep (G_i, H_i, term bound), position terms pushed to exact integer accumulators per "
                    "cell column, combine, dtheta reduction",
            "ms": round(t * 1e3, 3),
            "kernels": {k: {"launches": c // reps, "ms_per_call": round(ms_ / reps, 4)} for k, (c, ms_) in sorted(kt.items())}}


def jbar_measure(w, vct, L, nl, pos_s, cmap, perm, dev, reps=3):
    """The volume smoothing of the sigma method (Eq. VCT_bar_a) on the
    benchmark geometry (outside the timed steps): J = alpha of the mapping at
    every particle, Jbar^(N-1) = J scaled by seeded factors 1 + U(-0.05, 0.05),
    C_V = 1e-2 (dt x 10^2 with dt = 1e-4), r_e = R."""
    import numpy as np
    import torch
    from paper_2607_28872_amd import inputs as I
    progress("volume smoothing")
    n = w.n
    J = torch.empty(n, dtype=torch.float64, device=dev)
    vct.vct_map_alpha(w.dim, n, pos_s, cmap, J)
    fac = torch.as_tensor(I.volume_perturbation(n)[perm[:n].long().cpu().numpy()], device=dev)
    jb0 = J * fac
    ws = torch.empty(L.vct_jbar_workspace_size(n), dtype=torch.uint8, device=dev)
    jb = jb0.clone()
    vct.vct_jbar_smooth(nl, pos_s, J, jb, 1e-2, w.R, ws)   # warm-up
    torch.cuda.synchronize()
    vct.vct_timing_reset()
    vct.vct_timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        jb.copy_(jb0)
        vct.vct_jbar_smooth(nl, pos_s, J, jb, 1e-2, w.R, ws)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    vct.vct_timing_enable(False)
    kt = vct.vct_timing_read()
    vct.vct_timing_reset()
    v0 = float((J / jb0).sum().item())
    v1 = float((J / jb).sum().item())
    return {"what": "smoothed Jacobian determinant (Eq. VCT_bar_a), 27 colour phases of cells, C_V = 1e-2",
            "ms": round(t * 1e3, 3), "volume_drift": abs(v1 - v0) / v0,
            "kernels": {k: {"launches": c // reps, "ms_per_call": round(ms_ / reps, 4)} for k, (c, ms_) in sorted(kt.items())
                        if k.startswith("k_jbar")}}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, phis, mapspec, target_s):
    """The CPU oracle (neighbour search + SPH(2) operators, FP64, OpenMP) timed
    on a bounded sample of particles of the same set, on every host thread and
    on one; reported in evals/s.  Also returns the sampled rows and the
    oracle's records there, for the error report."""
    import numpy as np
    import oracle

    oracle.lib()
    nf = phis.shape[0]
    rng = np.random.default_rng(123)

    def timed(size, budget):
        while True:
            rows = np.sort(rng.choice(w.n, size=min(size, w.n), replace=False))
            t0 = time.perf_counter()
            csr = oracle.neighbors(w.pos, w.R, rows=rows)
            rec, _ = oracle.sph2(w.pos, w.vol, phis, w.kernel, w.R, mapspec, rows=rows, csr=csr)
            t = time.perf_counter() - t0
            if t >= budget / 4 or size >= w.n:
                return size, t, rows, rec
            size = int(min(w.n, size * max(2.0, 0.5 * budget / max(t, 1e-3))))

    cores = oracle.threads()
    size, t, rows, rec = timed(2000, target_s)
    oracle.set_threads(1)
    try:
        size1, t1, _, _ = timed(500, target_s / 3)
    finally:
        oracle.set_threads(cores)
    # per stage, on every thread: the neighbour search and the SPH(2)
    # operators at the sampled rows timed apart, and the adjoint d/dphi (each
    # sampled particle needs the Laplacian weights of its neighbours' rows)
    t0 = time.perf_counter()
    csr = oracle.neighbors(w.pos, w.R, rows=rows)
    t_nb = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.sph2(w.pos, w.vol, phis, w.kernel, w.R, mapspec, rows=rows, csr=csr)
    t_op = time.perf_counter() - t0
    u = rng.standard_normal(w.n)
    nadj = max(64, size // 200)
    ks = np.sort(rng.choice(w.n, size=min(nadj, w.n), replace=False))
    t0 = time.perf_counter()
    # the rows the sampled entries read: the sampled particles and their neighbours
    rp_k, col_k = oracle.neighbors(w.pos, w.R, rows=ks)
    need = np.unique(np.concatenate([ks, col_k.astype(np.int64)]))
    rp_n, col_n = oracle.neighbors(w.pos, w.R, rows=need)
    row_ptr = np.zeros(w.n + 1, dtype=np.int64)
    row_ptr[need + 1] = np.diff(rp_n)
    row_ptr = np.cumsum(row_ptr)
    oracle.adjoint_dphi(w.pos, w.vol, w.kernel, w.R, mapspec, u, ks=ks, csr=(row_ptr, col_n))
    t_adj = time.perf_counter() - t0
    res = {"value": size * nf / t, "unit": "evals/s", "cores": cores, "kind": "oracle",
           "sample": f"{size} random particles of the {w.n}-particle set (neighbour grid over all particles "
                     f"+ SPH(2) at the sampled rows), {t:.1f} s",
           "single_core": {"value": size1 * nf / t1, "sample": f"{size1} particles, {t1:.1f} s"},
           "per_stage": {
               "neighbours": {"particles_per_s": size / t_nb, "sample": f"{size} rows, {t_nb:.2f} s"},
               "moments_and_apply": {"particles_per_s": size * nf / t_op, "sample": f"{size} rows, {t_op:.2f} s"},
               "adjoint_dphi": {"particles_per_s": len(ks) / t_adj,
                                "sample": f"{len(ks)} particles (their neighbours' rows searched and re-evaluated), {t_adj:.2f} s"}},
           "cpu_model": cpu_model()}
    return res, rows, rec


def operator_errors(out_sampled, rec, dim):
    """Normwise error per output row (max |gpu - oracle| / max |oracle| over
    the sample, worst field) for the default rows: gradient, Laplacian, cross."""
    import numpy as np
    cols, names = ([0, 1, 2, 3, 4, 5, 6], ["grad_x", "grad_y", "grad_z", "lap", "cross_xy", "cross_xz", "cross_yz"]) \
        if dim == 3 else ([0, 2, 3, 5], ["grad_x", "grad_z", "lap", "cross_xz"])
    ref = np.transpose(rec[:, :, cols], (1, 0, 2))
    err = (np.abs(out_sampled - ref).max(axis=1) / np.abs(ref).max(axis=1)).max(axis=0)
    return {nm: float(f"{e:.3e}") for nm, e in zip(names, err)}


if __name__ == "__main__":
    main()
