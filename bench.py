#!/usr/bin/env python3
"""Benchmark of the DPLR long-range step (PPPM with ik-differentiation) on one GPU.

Workload: 72,192 rigid waters (216,576 atoms + 72,192 Wannier centroids,
288,768 charges) in a cubic 129.3 A box, beta = 0.4 1/A, mesh 128^3, B-spline
order 5, FP32 data path with FP64 influence table and FP64 energy/virial
reductions.  Each step evaluates energy, ion forces, WC forces and virial on
one frame of a seeded random walk (sigma = 0.02 A per coordinate per frame);
all frames are generated on the host and resident in HBM before timing.

  python bench.py [--steps K] [--warmup W] [--gpus 1]

Timed region: W warm-up steps, then exactly K steps replayed from a captured
HIP graph (one library call per step, one frame per step), bracketed by
torch.cuda.synchronize() on both sides.  A second pass runs the same K steps
eagerly with HIP events around every kernel (library instrumentation) to give
per-kernel durations for the roofline figure.  The CPU baseline times the FP64
Ewald oracle on a bounded sample (a same-density sub-box).

Prints one JSON line."""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "PPPM long-range ms/step & particles/s at 216k atoms; plain vs learned at force RMSE"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--order", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the order-8 and accuracy legs")
    ap.add_argument("--eager-only", action="store_true", help="no graph capture (profiling runs)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned coarse-mesh leg")
    ap.add_argument("--no-config5", action="store_true", help="skip the 1.2M-charge config-5 leg")
    ap.add_argument("--learned-boxes", type=int, default=2000, help="training boxes for the learned leg")
    ap.add_argument("--learned-epochs", type=int, default=3)
    ap.add_argument("--copy-ref-mb", type=float, default=0.0,
                    help="also run a plain device copy of this size (reference for rocprofv3 byte counters)")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter_collection.csv files (FETCH_SIZE, WRITE_SIZE) of a "
                         "--copy-ref-mb run into profiles/hbm_traffic.json, then exit")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_bytes(stage: str, N: int, K: int, order: int) -> float:
    """Algorithmic HBM bytes of one launch of a stage (FP32 plan, cubic mesh K^3):
    every array a kernel must read or write, read once and written once."""
    kh = K // 2 + 1
    spec = kh * K * K * 8           # complex64 half spectrum
    mesh_g = kh * (K // 2 + 1) ** 2 * 8  # FP64 influence table
    part = N * (16 + 4)             # sorted (d, q) float4 + packed stencil start
    if stage == "bin_count":
        return N * 12
    if stage == "bin_scatter":
        return N * (12 + 4) + N * (16 + 4 + 4)
    if stage in ("spread_fftx", "spread_xy"):
        # particles in, x- (or x- and y-) transformed half spectrum out
        return part + spec
    if stage == "ffty_fwd":
        return 2 * spec
    if stage == "fftz_poisson":
        return spec + mesh_g + 3 * spec
    if stage == "ffty_inv_reduce":
        return 2 * 3 * spec
    if stage == "ifftx":
        return 3 * spec + 3 * 4 * K ** 3
    if stage == "ifft_xy_reduce":
        # three field spectra in, interleaved real fields out
        return 3 * spec + 3 * 4 * K ** 3
    if stage == "gather":
        # fields read once + particles (d, q, stencil start, perm) + forces
        return 3 * 4 * K ** 3 + part + N * 4 + N * 12
    return 0.0


# kernel-name prefix -> stage name of the library instrumentation
KERNEL_STAGES = [("k_spread_xy", "spread_xy"), ("k_spread_fftx", "spread_fftx"), ("k_ffty<float, false>", "ffty_fwd"),
                 ("k_fftz_poisson", "fftz_poisson"), ("k_ffty<float, true>", "ffty_inv_reduce"),
                 ("k_ifftx", "ifftx"), ("k_ifft_xy", "ifft_xy_reduce"), ("k_gather", "gather"), ("k_bin_hist", "bin_count"),
                 ("k_bin_place", "bin_scatter"), ("k_bin_colscan", "bin_scan")]


def ingest_counters(fetch_csv: str, write_csv: str, copy_mb: float) -> dict:
    """Per-launch HBM-side bytes of every kernel of the benchmark step from two
    rocprofv3 counter runs (FETCH_SIZE and WRITE_SIZE, KiB per dispatch), each
    scaled by what the same counter reads for a plain copy of copy_mb MB."""
    import csv
    import statistics

    def load(path, counter):
        per, copies = {}, []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            name, val = r["Kernel_Name"], float(r["Counter_Value"]) * 1024.0
            per.setdefault(name, []).append(val)
            if "copy" in name.lower():
                copies.append((name, val))
        return per, copies

    copy_bytes = copy_mb * 1e6

    def scale(copies):
        # the reference copy's dispatches: the copy-kernel dispatches within 2x of its size
        near = [v for _, v in copies if 0.5 * copy_bytes <= v <= 2.0 * copy_bytes]
        if not near:
            raise RuntimeError("no copy dispatch of the reference size in the counter run (use --copy-ref-mb)")
        return statistics.median(near) / copy_bytes, next(n for n, v in copies if v in near)

    (fetch, fc), (write, wc) = load(fetch_csv, "FETCH_SIZE"), load(write_csv, "WRITE_SIZE")
    f_scale, ck = scale(fc)
    w_scale, _ = scale(wc)
    out = {"source_digest": source_digest(), "copy_kernel": ck.split("(")[0], "copy_mb": copy_mb,
           "fetch_scale": f_scale, "write_scale": w_scale, "kernels": {}}
    for name, vals in fetch.items():
        stage = next((st for pre, st in KERNEL_STAGES if pre in name), None)
        if stage is None:
            continue
        wv = write.get(name, [0.0])
        fb = statistics.median(vals) / f_scale
        wb = statistics.median(wv) / w_scale
        rec = out["kernels"].setdefault(stage, {"fetch_bytes": 0.0, "write_bytes": 0.0, "bytes_per_launch": 0.0})
        # several kernels can share a stage (the scans): add them
        rec["fetch_bytes"] += fb
        rec["write_bytes"] += wb
        rec["bytes_per_launch"] = rec["fetch_bytes"] + rec["write_bytes"]
    return out


def source_digest() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2504_15508_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(stage: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_digest") != source_digest():
        return None
    k = d.get("kernels", {}).get(stage)
    return None if k is None else float(k["bytes_per_launch"])


def cpu_baseline():
    """The FP64 Ewald oracle timed on a bounded sample of the workload: the same
    water recipe and density on a cubic box of half the volume (36,096 waters,
    144,384 charges, 102.6 A), energy + all forces + virial."""
    import numpy as np
    import systems
    from oracle import ewald
    ewald.build(force=False)
    n_w = 72192 // 2
    s = systems.water_box(n_w, 129.3 / 2 ** (1 / 3), seed=systems.SEED_BASE + 3).rounded(np.float32)
    t = time.perf_counter()
    ewald.recip(s.all_pos(), s.all_q(), s.box, systems.BETA, systems.COULOMB_K)
    dt = time.perf_counter() - t
    return {"value": s.n / dt, "unit": "particles/s", "cores": int(ewald.threads_used()), "kind": "oracle",
            "seconds": dt,
            "sample": "FP64 direct Ewald (energy, all forces, virial) on 36,096 waters (144,384 charges) in a "
                      "102.6 A cubic box: the benchmark's recipe and density at half its volume; the direct sum "
                      "costs O(N^2) at fixed density, so the full 288,768-charge system takes ~4x longer in total "
                      "and ~2x longer per charge"}


def cpu_pppm_oracle():
    """The like-for-like CPU figure: the NumPy FP64 PPPM oracle (the same
    discrete operator as the GPU path: spread, FFTs, influence multiply with
    ik, three inverse FFTs, gather) on the full benchmark system (288,768
    charges, 128^3, order 5), one step, single process.  The per-box influence
    table is computed first and not timed (the GPU computes it per box too)."""
    import numpy as np
    import systems
    from oracle import pppm
    w = systems.workload(3)
    s = w.system().rounded(np.float32)
    G = pppm.influence(s.box, (w.mesh,) * 3, w.beta, w.order)
    t = time.perf_counter()
    pppm.pppm(s.all_pos(), s.all_q(), s.box, (w.mesh,) * 3, w.order, w.beta, w.coulomb_k, G=G)
    dt = time.perf_counter() - t
    return {"value": s.n / dt, "unit": "particles/s", "cores": 1, "kind": "oracle", "seconds": dt,
            "sample": "FP64 NumPy PPPM oracle (ik, order 5, 128^3), one full step of the benchmark system "
                      "(288,768 charges), single process; influence table precomputed"}


# The paper's own speeds (whole DPLR MD steps on Fugaku A64FX, not the
# long-range step alone): context, not a target.
PAPER_CONTEXT = [
    {"ns_per_day": 51.0, "nodes": 12, "machine": "Fugaku (A64FX), 4 MPI ranks per node",
     "system": "564-atom water", "what": "whole DPLR MD step (peak speed)"},
    {"ns_per_day": 32.5, "nodes": 8400, "machine": "Fugaku (A64FX)",
     "system": "about 400,000-atom water (20 x 21 x 20 replication)", "what": "whole DPLR MD step (weak scaling)"},
    {"ns_per_day": 37.0, "nodes": 4608, "machine": "Fugaku (A64FX)",
     "system": "216,576-atom water (16 x 18 x 16 replication)",
     "what": "whole DPLR MD step; appears only in a commented-out draft of the abstract"},
]


def overlap_leg(plan, step, W, K, n_atoms, energy, dev):
    """Single-GPU analogue of the paper's overlap of the long-range step with
    the short-range networks: the step's graph replays on its own stream while
    a stand-in short-range workload replays on another.  The stand-in is a
    per-atom bf16 MLP (128 -> 256 -> 256 -> 1, SiLU) forward plus the backward
    to its inputs (four GEMMs), synthetic weights and inputs.  Returns the
    step time of each alone and of both together, and whether the overlapped
    long-range results equal the isolated ones bitwise."""
    import torch
    import torch.nn.functional as Fn
    g = torch.Generator(device=dev).manual_seed(7)
    D, H = 128, 256
    X = torch.randn(n_atoms, D, device=dev, generator=g).bfloat16()
    W1 = (torch.randn(D, H, device=dev, generator=g) / D ** 0.5).bfloat16()
    W2 = (torch.randn(H, H, device=dev, generator=g) / H ** 0.5).bfloat16()
    w3 = (torch.randn(H, device=dev, generator=g) / H ** 0.5).bfloat16()
    W1t, W2t = W1.t().contiguous(), W2.t().contiguous()
    gX = torch.empty(n_atoms, D, device=dev, dtype=torch.bfloat16)

    def sr():
        z1 = X @ W1
        z2 = Fn.silu(z1) @ W2
        s2 = torch.sigmoid(z2)
        gz2 = w3 * s2 * (1 + z2 * (1 - s2))          # d e / d z2, e = silu(z2) . w3
        ga1 = gz2 @ W2t
        s1 = torch.sigmoid(z1)
        torch.matmul(ga1 * s1 * (1 + z1 * (1 - s1)), W1t, out=gX)

    s_lr, s_sr = torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)
    with torch.cuda.stream(s_lr):
        step(plan, 0)                                 # binds the plan to its stream
    with torch.cuda.stream(s_sr):
        sr()
    torch.cuda.synchronize()
    g_lr, g_sr = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    with torch.cuda.graph(g_lr, stream=s_lr):
        for t in range(W, W + K):
            step(plan, t)
    with torch.cuda.graph(g_sr, stream=s_sr):
        for _ in range(K):
            sr()

    def run(lr, sr_on):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if lr:
            with torch.cuda.stream(s_lr):
                g_lr.replay()
        if sr_on:
            with torch.cuda.stream(s_sr):
                g_sr.replay()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / K

    run(True, True)
    t_lr = run(True, False)
    e_alone = energy[W:W + K].clone()
    t_sr = run(False, True)
    t_both = run(True, True)
    same = bool(torch.equal(energy[W:W + K], e_alone))
    return {"overlap_lr_ms_per_step": 1e3 * t_lr, "overlap_sr_ms_per_step": 1e3 * t_sr,
            "overlap_both_ms_per_step": 1e3 * t_both,
            "overlap_hidden_frac_of_lr": (t_lr + t_sr - t_both) / t_lr,
            "overlap_lr_bitwise_equal": same,
            "overlap_sr_stand_in": "per-atom bf16 MLP 128-256-256-1 (SiLU), forward + input gradient, "
                                   f"{n_atoms} atoms"}


def step_percentiles(plan, step, W, K, dev):
    """Median, p10 and p90 of the per-frame step time: each of the K timed
    frames captured in a graph of its own, replayed between HIP events (GPU
    time of the step without host launch gaps)."""
    import numpy as np
    import torch

    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        step(plan, 0)
    torch.cuda.synchronize()
    graphs = []
    for t in range(W, W + K):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            step(plan, t)
        graphs.append(g)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in graphs]
    with torch.cuda.stream(stream):
        for g, (a, b) in zip(graphs, ev):
            a.record(stream)
            g.replay()
            b.record(stream)
    torch.cuda.synchronize()
    ms = np.array([a.elapsed_time(b) for a, b in ev])
    del graphs
    return {"p10": float(np.percentile(ms, 10)), "median": float(np.median(ms)),
            "p90": float(np.percentile(ms, 90)), "frames": int(K)}


def mixed_leg(args, make_plan, step, timed_graph, timed_eager, s0, qi, qw, w, dev):
    """The mixed-radix kernels: the same 216,576 + 72,192 charges on a 120^3
    mesh (h = 1.078 A, next to the 128^3 of the headline), and the paper's
    12x18x12 precision-study grid (128 waters, 16 A) with exact and with
    int32-quantised transforms."""
    import numpy as np
    import torch
    import systems
    import paper_2504_15508_amd as dl

    out = {}
    gpath = os.path.join(ROOT, "tests", "golden", f"ewald_{w.name}.json")
    p = make_plan(args.order, mesh=(120, 120, 120))
    if os.path.exists(gpath):
        gold = json.load(open(gpath))
        idx = np.array(gold["sample_index"])
        fref = np.array(gold["sample_force"])
        r0 = torch.tensor(s0.ion_pos, dtype=torch.float32, device=dev)
        w0 = torch.tensor(s0.wc_pos, dtype=torch.float32, device=dev)
        E, a, b, _ = p.compute(r0, qi, w0, qw)
        F = torch.cat([a, b]).double().cpu().numpy()[idx]
        out["mixed120_force_rmse_vs_ewald"] = float(np.linalg.norm(F - fref) / np.linalg.norm(fref))
    if args.eager_only:
        out["mixed120_ms_per_step"] = 1e3 * timed_eager(p, False)[0]
    else:
        out["mixed120_ms_per_step"] = 1e3 * timed_graph(lambda t: step(p, t))
        _, prof = timed_eager(p, True)
        out["mixed120_kernels_us"] = {k: round(1e3 * v[0] / max(v[1], 1), 2) for k, v in prof.items() if v[1]}
    p.close()
    # the paper's grid: eleven small kernels; eager calls on one frame
    sm = systems.water_box(128, 16.0, seed=20261128)
    t = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=torch.float32, device=dev)
    args_sm = (t(sm.ion_pos), t(sm.ion_q), t(sm.wc_pos), t(sm.wc_q))
    for tag, nodes in (("grid12x18x12", None), ("grid12x18x12_int32", (2, 3, 2))):
        ps = dl.Plan((12, 18, 12), order=5, beta=w.beta, coulomb_k=w.coulomb_k, precision="fp32", capacity=sm.n)
        ps.set_box(sm.box)
        if nodes:
            ps.set_fft_int32(nodes, 1e7)
        for _ in range(5):
            ps.compute(*args_sm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(50):
            ps.compute(*args_sm)
        torch.cuda.synchronize()
        out[f"{tag}_ms_per_call"] = 1e3 * (time.perf_counter() - t0) / 50
        if not args.eager_only:
            # 50 calls captured in one graph: the launch overhead removed
            stream = torch.cuda.Stream(device=dev)
            with torch.cuda.stream(stream):
                ps.compute(*args_sm)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=stream):
                for _ in range(50):
                    ps.compute(*args_sm)
            g.replay()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.replay()
            torch.cuda.synchronize()
            out[f"{tag}_graph_ms_per_call"] = 1e3 * (time.perf_counter() - t0) / 50
        ps.close()
    return out


def learned_leg(args, w, s0, ion_d, wc_d, qi, qw, dev, timed_graph_fn, plain_ms, gold):
    """Learned coarse form: train the correction on spacing-matched boxes
    (1,128 waters in 32.325 A, meshes 16^3 / 32^3 = the spacings of 64^3 /
    128^3 here), then evaluate 64^3 + correction on frame 0 against the stored
    Ewald forces and time it as the plain step is timed."""
    import numpy as np
    import torch
    import systems
    import paper_2504_15508_amd as dl
    from paper_2504_15508_amd import learned as L

    t0 = time.perf_counter()
    boxes = [systems.training_box(i) for i in range(args.learned_boxes)]
    held = [systems.training_box(i, heldout=True) for i in range(max(1, args.learned_boxes // 10))]
    log(f"learned leg: training on {len(boxes)} boxes x {args.learned_epochs} epochs")
    mlp = L.Mlp(s0.n, device=dev)
    mlp, rep = L.train(boxes, held, coarse_mesh=16, fine_mesh=32, epochs=args.learned_epochs, lr=2e-3, mlp=mlp,
                       device=dev, log=lambda m: log("  " + m))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del boxes, held

    coarse = dl.Plan(w.coarse_mesh, order=w.order, beta=w.beta, coulomb_k=w.coulomb_k, precision="fp32",
                     capacity=s0.n, device=dev)
    coarse.set_box(s0.box)
    fine = dl.Plan(w.mesh, order=w.order, beta=w.beta, coulomb_k=w.coulomb_k, precision="fp32",
                   capacity=s0.n, device=dev)
    fine.set_box(s0.box)
    r0 = torch.tensor(s0.ion_pos, dtype=torch.float32, device=dev)
    w0 = torch.tensor(s0.wc_pos, dtype=torch.float32, device=dev)
    out = {"learned_train_boxes": args.learned_boxes, "learned_train_epochs": args.learned_epochs,
           "learned_train_seconds": train_s,
           "learned_heldout_rel_rmse_vs_fine": rep.heldout_rel_rmse_learned,
           "coarse_heldout_rel_rmse_vs_fine": rep.heldout_rel_rmse_coarse}
    idx = np.array(gold["sample_index"]) if gold else None
    fref = np.array(gold["sample_force"]) if gold else None

    def rmse(a, b):
        F = torch.cat([a, b]).double().cpu().numpy()[idx]
        return float(np.linalg.norm(F - fref) / np.linalg.norm(fref))

    _, ci, cw, _ = coarse.compute(r0, qi, w0, qw)
    ci, cw = ci.clone(), cw.clone()
    di, dw = mlp.forward(s0.box, r0, qi, w0, qw)
    if gold:
        out["coarse64_force_rmse_vs_ewald"] = rmse(ci, cw)
        out["learned64_force_rmse_vs_ewald"] = rmse(ci + di, cw + dw)
    # guarded driver: first call audits against the 128^3 plan
    lc = L.LearnedCoarse(s0.box, coarse, fine, mlp, guard_cfg=dict(max_audit_rel_rmse=1e-3))
    modes = [lc.compute(r0, qi, w0, qw)[4] for _ in range(2)]
    out["learned_audit_rel_rmse_vs_128"] = lc.stats["audit_rel_rmse"]
    out["learned_guard_modes"] = modes

    # timing: coarse plan + descriptor + network, one captured graph per K steps
    fi = torch.empty((s0.n_ion, 3), dtype=torch.float32, device=dev)
    fw = torch.empty((s0.n_wc, 3), dtype=torch.float32, device=dev)
    e = torch.empty((), dtype=torch.float64, device=dev)
    v = torch.empty(6, dtype=torch.float64, device=dev)

    def lstep(t):
        coarse.compute(ion_d[t], qi, wc_d[t], qw, ion_force=fi, wc_force=fw, energy=e, virial=v)
        mlp.forward(s0.box, ion_d[t], qi, wc_d[t], qw, fi, fw, accumulate=True)

    def cstep(t):
        coarse.compute(ion_d[t], qi, wc_d[t], qw, ion_force=fi, wc_force=fw, energy=e, virial=v)

    # learned mode itself (coarse plan + descriptor + network every step; the
    # guard's audits and fallbacks are timed by the plain legs)
    out["learned64_ms_per_step"] = 1e3 * timed_graph_fn(lstep)
    out["coarse64_ms_per_step"] = 1e3 * timed_graph_fn(cstep)
    out["plain128_ms_per_step"] = plain_ms
    coarse.close()
    fine.close()
    mlp.close()
    return out


def config5_leg(args, dev, timed_steps):
    """The heterogeneous ionic solution (300,000 waters + 3,000 Na+ + 3,000
    Cl-, 1,206,000 charges, 208.5 A): the plain step at 256^3 against the
    coarse 128^3 step with the network correction (descriptor + MLP), each
    with the autograd backward (dE/dr = -g F) per step, on the same
    random-walk frames.  The network is untrained (its cost does not depend
    on its weights); the accuracy side is the learned leg's."""
    import numpy as np
    import torch
    import systems
    import paper_2504_15508_amd as dl
    from paper_2504_15508_amd import learned as L
    w = systems.workload(5)
    s = w.system()
    nf = 4
    rng = np.random.Generator(np.random.PCG64(w.seed + 7))
    ion = np.empty((nf, s.n_ion, 3), np.float32)
    wc = np.empty((nf, s.n_wc, 3), np.float32)
    fi, fw = s.ion_pos.copy(), s.wc_pos.copy()
    for t in range(nf):
        ion[t], wc[t] = fi, fw
        fi = np.mod(fi + rng.normal(0, 0.02, fi.shape), s.box)
        fw = np.mod(fw + rng.normal(0, 0.02, fw.shape), s.box)
    ion_d, wc_d = torch.from_numpy(ion).to(dev), torch.from_numpy(wc).to(dev)
    qi = torch.tensor(s.ion_q, dtype=torch.float32, device=dev)
    qw = torch.tensor(s.wc_q, dtype=torch.float32, device=dev)
    f_i = torch.empty((s.n_ion, 3), dtype=torch.float32, device=dev)
    f_w = torch.empty((s.n_wc, 3), dtype=torch.float32, device=dev)
    g_i, g_w = torch.empty_like(f_i), torch.empty_like(f_w)
    e = torch.empty((), dtype=torch.float64, device=dev)
    v = torch.empty(6, dtype=torch.float64, device=dev)
    one = torch.ones((), dtype=torch.float64, device=dev)
    plain = dl.Plan(w.mesh, order=w.order, beta=w.beta, coulomb_k=w.coulomb_k, precision="fp32", capacity=s.n)
    plain.set_box(s.box)
    coarse = dl.Plan(w.coarse_mesh, order=w.order, beta=w.beta, coulomb_k=w.coulomb_k, precision="fp32",
                     capacity=s.n)
    coarse.set_box(s.box)
    mlp = L.Mlp(s.n, device=dev)
    mlp.set_params(L.init_params(0))

    def pstep(t):
        plain.compute(ion_d[t % nf], qi, wc_d[t % nf], qw, ion_force=f_i, wc_force=f_w, energy=e, virial=v)
        plain.scale_grad(one, f_i, f_w, g_i, g_w)

    def lstep(t):
        coarse.compute(ion_d[t % nf], qi, wc_d[t % nf], qw, ion_force=f_i, wc_force=f_w, energy=e, virial=v)
        mlp.forward(s.box, ion_d[t % nf], qi, wc_d[t % nf], qw, f_i, f_w, accumulate=True)
        coarse.scale_grad(one, f_i, f_w, g_i, g_w)

    def cstep(t):
        coarse.compute(ion_d[t % nf], qi, wc_d[t % nf], qw, ion_force=f_i, wc_force=f_w, energy=e, virial=v)
        coarse.scale_grad(one, f_i, f_w, g_i, g_w)

    out = {"config5_particles": s.n,
           "config5_plain256_fwd_bwd_ms_per_step": 1e3 * timed_steps(pstep),
           "config5_coarse128_fwd_bwd_ms_per_step": 1e3 * timed_steps(cstep),
           "config5_learned128_fwd_bwd_ms_per_step": 1e3 * timed_steps(lstep)}
    plain.close()
    coarse.close()
    mlp.close()
    return out


def main():
    args = parse()
    if args.ingest_counters:
        out = ingest_counters(args.ingest_counters[0], args.ingest_counters[1], args.copy_ref_mb or 256.0)
        path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
        with open(path, "w") as fh:
            json.dump(out, fh, indent=1)
        print(json.dumps(out))
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; run with --gpus 1.",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch
    import systems
    import paper_2504_15508_amd as dl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    w = systems.workload(3)
    s0 = w.system()
    K, W = args.steps, args.warmup
    log(f"generating {W + K} frames of {s0.n} charges")
    rng = np.random.Generator(np.random.PCG64(w.seed + 7))
    ion = np.empty((W + K, s0.n_ion, 3), np.float32)
    wc = np.empty((W + K, s0.n_wc, 3), np.float32)
    fi, fw = s0.ion_pos.copy(), s0.wc_pos.copy()
    for t in range(W + K):
        ion[t], wc[t] = fi, fw
        fi = np.mod(fi + rng.normal(0, 0.02, fi.shape), s0.box)
        fw = np.mod(fw + rng.normal(0, 0.02, fw.shape), s0.box)
    ion_d = torch.from_numpy(ion).to(dev)
    wc_d = torch.from_numpy(wc).to(dev)
    qi = torch.tensor(s0.ion_q, dtype=torch.float32, device=dev)
    qw = torch.tensor(s0.wc_q, dtype=torch.float32, device=dev)
    N = s0.n

    def make_plan(order, mesh=w.mesh, diff="ik"):
        p = dl.Plan(mesh, order=order, beta=w.beta, coulomb_k=w.coulomb_k, precision="fp32", capacity=N, diff=diff)
        p.set_box(s0.box)
        return p

    plan = make_plan(args.order)
    f_ion = torch.empty((s0.n_ion, 3), dtype=torch.float32, device=dev)
    f_wc = torch.empty((s0.n_wc, 3), dtype=torch.float32, device=dev)
    energy = torch.empty((W + K,), dtype=torch.float64, device=dev)
    virial = torch.empty((W + K, 6), dtype=torch.float64, device=dev)

    def step(p, t):
        p.compute(ion_d[t], qi, wc_d[t], qw, ion_force=f_ion, wc_force=f_wc, energy=energy[t], virial=virial[t])

    def timed_graph(fn):
        """K steps fn(W), ..., fn(W + K - 1) replayed from one captured graph."""
        stream = torch.cuda.Stream(device=dev)
        torch.cuda.synchronize()
        gw, gt = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
        with torch.cuda.stream(stream):
            fn(0)                    # binds the plans to the capture stream outside capture
        torch.cuda.synchronize()
        with torch.cuda.graph(gw, stream=stream):
            for t in range(W):
                fn(t)
        with torch.cuda.graph(gt, stream=stream):
            for t in range(W, W + K):
                fn(t)
        gw.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gt.replay()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / K

    def timed_eager(p, profile):
        for t in range(W):
            step(p, t)
        torch.cuda.synchronize()
        p.profile(profile)
        if profile:
            p.profile_read(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(W, W + K):
            step(p, t)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / K
        prof = p.profile_read(reset=True) if profile else {}
        p.profile(False)
        return dt, prof

    result = {}
    if args.copy_ref_mb > 0:
        nb = int(args.copy_ref_mb * 1e6 / 4)
        xs = torch.ones(nb, dtype=torch.float32, device=dev)
        ys = torch.empty_like(xs)
        for _ in range(3):
            ys.copy_(xs)
        torch.cuda.synchronize()
        del xs, ys
    if args.eager_only:
        sec = None
    else:
        log("timed region: graph replay")
        sec = timed_graph(lambda t: step(plan, t))
    pct = None
    if not args.eager_only:
        log("per-frame graphs: step time percentiles")
        pct = step_percentiles(plan, step, W, K, dev)
    log("eager pass with per-kernel HIP events")
    eager_sec, prof = timed_eager(plan, True)
    if sec is None:
        sec = eager_sec
    ms = sec * 1e3
    kernels = {k: {"avg_us": 1e3 * v[0] / max(v[1], 1), "launches": v[1],
                   "alg_bytes": kernel_bytes(k, N, w.mesh, args.order)} for k, v in prof.items() if v[1]}
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"])
    kd = kernels[dom]
    achieved = kd["alg_bytes"] / (kd["avg_us"] * 1e-6) / 1e9
    traffic = measured_traffic(dom)
    step_bytes = sum(v["alg_bytes"] * v["launches"] for v in kernels.values()) / K

    extras = {}
    if not args.no_extras:
        try:
            # accuracy on frame 0 against stored Ewald values (if present)
            gpath = os.path.join(ROOT, "tests", "golden", f"ewald_{w.name}.json")
            if os.path.exists(gpath):
                gold = json.load(open(gpath))
                idx = np.array(gold["sample_index"])
                fref = np.array(gold["sample_force"])
                # ik at the benchmark's order and at order 8; analytic differentiation at both
                for order, diff in sorted({(args.order, "ik"), (7, "ik"), (8, "ik"), (args.order, "ad"), (8, "ad")}):
                    own = order == args.order and diff == "ik"
                    p = plan if own else make_plan(order, diff=diff)
                    tag = f"order{order}" if diff == "ik" else f"ad{order}"
                    r0 = torch.tensor(s0.ion_pos, dtype=torch.float32, device=dev)
                    w0 = torch.tensor(s0.wc_pos, dtype=torch.float32, device=dev)
                    E, a, b, Wv = p.compute(r0, qi, w0, qw)
                    F = torch.cat([a, b]).double().cpu().numpy()[idx]
                    extras[f"{tag}_force_rmse_vs_ewald"] = float(np.linalg.norm(F - fref) / np.linalg.norm(fref))
                    extras[f"{tag}_energy_relerr_vs_ewald"] = abs(float(E) - gold["energy"]) / abs(gold["energy"])
                    if not own:
                        extras[f"{tag}_ms_per_step"] = 1e3 * (timed_graph(lambda t: step(p, t)) if not args.eager_only
                                                              else timed_eager(p, False)[0])
                        p.close()
                # the FP64 plan: the same step in FP64 throughout (FP64 frames)
                p = dl.Plan(w.mesh, order=args.order, beta=w.beta, coulomb_k=w.coulomb_k, precision="fp64",
                            capacity=N)
                p.set_box(s0.box)
                ion64, wc64 = ion_d.double(), wc_d.double()
                qi64, qw64 = qi.double(), qw.double()
                fi64 = torch.empty((s0.n_ion, 3), dtype=torch.float64, device=dev)
                fw64 = torch.empty((s0.n_wc, 3), dtype=torch.float64, device=dev)

                def step64(t):
                    p.compute(ion64[t], qi64, wc64[t], qw64, ion_force=fi64, wc_force=fw64, energy=energy[t],
                              virial=virial[t])
                E, a, b, _ = p.compute(ion64[0], qi64, wc64[0], qw64)
                F = torch.cat([a, b]).cpu().numpy()[idx]
                extras["fp64_force_rmse_vs_ewald"] = float(np.linalg.norm(F - fref) / np.linalg.norm(fref))
                extras["fp64_ms_per_step"] = 1e3 * (timed_graph(step64) if not args.eager_only
                                                    else timed_eager(p, False)[0])
                p.close()
                del ion64, wc64
        except Exception as e:  # extras never hide the headline measurement
            extras["extras_error"] = repr(e)
    if not args.no_extras:
        try:
            extras.update(mixed_leg(args, make_plan, step, timed_graph, timed_eager, s0, qi, qw, w, dev))
        except Exception as e:
            extras["mixed_error"] = repr(e)
    if not args.no_extras and not args.eager_only:
        try:
            extras.update(overlap_leg(plan, step, W, K, s0.n_ion, energy, dev))
        except Exception as e:
            extras["overlap_error"] = repr(e)
    if not args.no_learned and not args.eager_only:
        try:
            gpath = os.path.join(ROOT, "tests", "golden", f"ewald_{w.name}.json")
            gold = json.load(open(gpath)) if os.path.exists(gpath) else None
            extras.update(learned_leg(args, systems.workload(4), s0, ion_d, wc_d, qi, qw, dev, timed_graph, ms,
                                      gold))
        except Exception as e:
            extras["learned_error"] = repr(e)

    if not args.no_learned and not args.no_config5 and not args.eager_only:
        try:
            log("config-5 leg: 1,206,000 charges, 256^3 plain vs 128^3 + network")
            extras.update(config5_leg(args, dev, timed_graph))
        except Exception as e:
            extras["config5_error"] = repr(e)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline()
        log("cpu PPPM oracle (NumPy, one full step)")
        extras["cpu_pppm_oracle"] = cpu_pppm_oracle()

    out = {
        "metric": METRIC,
        "value": N / sec,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "water72192_fp32: 216,576 atoms + 72,192 WCs, 129.3 A cubic box, "
                               "beta 0.4, mesh 128^3, order %d, FP32 (FP64 influence table and reductions), "
                               "random-walk frames sigma 0.02 A" % args.order,
                   "particles": N, "atoms": s0.n_ion, "wcs": s0.n_wc, "mesh": w.mesh, "order": args.order},
        "atoms_per_s": s0.n_ion / sec,
        "eager_ms_per_step": eager_sec * 1e3,
        "step_ms_percentiles": pct,
        "step_alg_bytes": step_bytes,
        "step_roofline_frac": step_bytes / sec / 1e9 / HBM_PEAK_GBS,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        # every kernel of the step against the same peak, by name (the
        # target is a fraction of 0.5 for the step)
        "roofline_by_kernel": {k: {"achieved_gbs": v["alg_bytes"] / (v["avg_us"] * 1e-6) / 1e9,
                                   "frac": v["alg_bytes"] / (v["avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS,
                                   "traffic": measured_traffic(k)} for k, v in kernels.items()},
        "roofline_target_frac": 0.5,
        "kernels": kernels,
        "cpu_baseline": cpu,
        "paper_context": PAPER_CONTEXT,
        "source_digest": source_digest(),
    }
    out.update(extras)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
