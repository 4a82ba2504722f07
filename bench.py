"""Benchmark: pseudo-time steps of the 256^3 FP64 cavity on one MI355X.

One step = halo pack + halo unpack of the 3D (2,2,2) virtual split +
residual/update sweep (wall ghosts derived inside it) with the centre
rescale; the residual norms are reduced on the last step.  That is one
GPU's share of an iteration of the paper's solver (Xue & Roy,
arXiv:2006.02602, Sec. 3.1 and 4.5).  Also reported: halo pack/unpack per
split and width pattern, and the FP32 precision form (384^3).
Inputs are seeded synthetic fields already resident in HBM.  Prints ONE JSON
line; `value` is interior grid-point updates per second.

    python bench.py [--gpus 1] [--steps 200] [--warmup 20] [--no-cpu]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak
SWEEP_BYTES_PER_CELL = 80      # read 5 + write 5 FP64 fields per interior cell
ADJ_MIN_BYTES_PER_CELL = 120   # reverse step: read q^n and lambda, write lambda (5 FP64 fields each)
PAPER_SSSPNT_P100 = 93.8       # single-GPU row of Tables 3-4 (P100, 256^3, no halo)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sweep_source_hash():
    h = hashlib.sha256()
    for f in ("sweep.hip", "sweep_tile.h", "stencil.h", "cavity_internal.h"):
        with open(os.path.join(ROOT, "paper_2006_02602_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(kernel_hash):
    """HBM bytes per sweep launch from the committed rocprofv3 counter
    summary, if it was taken on the current sweep source; else None."""
    path = os.path.join(ROOT, "profiles", "sweep_cavity256_f64_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"sweep source hash:\s*`?([0-9a-f]+)", text)
    m_bytes = re.search(r"calibrated HBM bytes per sweep launch:\s*([0-9.eE+]+)", text)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_hash:
        return None
    return float(m_bytes.group(1))


def f32_batch_counter_bytes():
    """HBM bytes (read + write) per launch of the 384^3 FP32 sweep and per
    batch step, from the committed rocprofv3 counter summary, if it was taken
    on the current sweep source; else {}."""
    path = os.path.join(ROOT, "profiles", "sweep_f32_batch_counters.md")
    if not os.path.exists(path):
        return {}
    text = open(path).read()
    m = re.search(r"sweep source hash:\s*`?([0-9a-f]+)", text)
    if not m or m.group(1) != sweep_source_hash():
        return {}
    out = {}
    for line in text.splitlines():
        c = [x.strip() for x in line.strip().strip("|").split("|")]
        if len(c) < 3:
            continue
        key = ("f32_sweep" if c[0].startswith("`sweep_kernel<float, false") else
               "batch" if c[0].startswith("`batch_kernel<float, false") else None)
        if key:
            out[key] = float(c[1]) + float(c[2])
    return out


def adjoint_source_hash():
    h = hashlib.sha256()
    for f in ("adjoint.hip", "sweep_tile.h", "stencil.h", "cavity_internal.h"):
        with open(os.path.join(ROOT, "paper_2006_02602_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def adjoint_counter_bytes():
    """HBM bytes per 256^3 reverse step from the committed rocprofv3 counter
    summary, if it was taken on the current adjoint source; else None."""
    path = os.path.join(ROOT, "profiles", "adjoint_cavity256_f64_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"adjoint source hash[^`]*`([0-9a-f]+)`", text)
    m_bytes = re.search(r"calibrated HBM bytes per 256\^3 reverse step[^:]*:\s*([0-9.eE+]+)", text)
    if not m_hash or not m_bytes or m_hash.group(1) != adjoint_source_hash():
        return None
    return float(m_bytes.group(1))


def halo_source_hash():
    h = hashlib.sha256()
    for f in ("halo.hip", "halo_layout.h"):
        with open(os.path.join(ROOT, "paper_2006_02602_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def halo_counter_bytes():
    """HBM bytes (read + write) per pack/unpack launch by split, widths,
    mode and kernel, from the committed rocprofv3 counter summary, if it was
    taken on the current halo source; else {}."""
    path = os.path.join(ROOT, "profiles", "halo_pack_unpack_cavity256_f64_counters.md")
    if not os.path.exists(path):
        return {}
    text = open(path).read()
    m = re.search(r"halo source hash[^`]*`([0-9a-f]+)`", text)
    if not m or m.group(1) != halo_source_hash():
        return {}
    out = {}
    for line in text.splitlines():
        c = [x.strip() for x in line.strip().strip("|").split("|")]
        if len(c) < 9 or not re.fullmatch(r"\d+x\d+x\d+", c[0]):
            continue
        try:
            out[(c[0], c[1].replace(" ", ""), c[2], c[3])] = float(c[7]) + float(c[8])
        except ValueError:
            continue
    return out


def halo_bench(C, torch, grid, cav, splits, widths_list, reps):
    """Warm and cold (after a 1 GiB flush write) pack/unpack timings."""
    out = []
    counted = halo_counter_bytes()
    flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    for split in splits:
        for widths in widths_list:
            h = C.Halo(split, widths)
            nbytes = C.halo_buffer_bytes(grid, h)
            buf = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
            elems = nbytes // 8
            res = {"split": list(split), "widths": list(widths), "values": elems}
            for mode in ("warm", "cold"):
                C.cavity_timing_read()
                torch.cuda.synchronize()
                for _ in range(reps):
                    if mode == "cold":
                        flush.zero_()
                    C.cavity_timing_enable(True)
                    C.halo_pack(grid, h, cav.q, buf)
                    C.halo_unpack(grid, h, buf, cav.q)
                    C.cavity_timing_enable(False)
                torch.cuda.synchronize()
                kt = C.cavity_timing_read()
                for k in ("halo_pack", "halo_unpack"):
                    n, ms = kt[k]
                    us = 1e3 * ms / n
                    res["%s_%s_us" % (k.split("_")[1], mode)] = round(us, 2)
                    res["%s_%s_GBs" % (k.split("_")[1], mode)] = round(16.0 * elems / (us * 1e-6) / 1e9, 1)
                    key = ("x".join(map(str, split)), ",".join(map(str, widths)), mode, k.split("_")[1])
                    if key in counted:
                        # HBM bytes by the counters (profiles/) over this run's launch time
                        gbs = counted[key] / (us * 1e-6) / 1e9
                        res["%s_%s_counter_GBs" % (k.split("_")[1], mode)] = round(gbs, 1)
                        res["%s_%s_counter_frac" % (k.split("_")[1], mode)] = round(gbs / HBM_PEAK_GBS, 3)
            out.append(res)
            del buf
    del flush
    return out


def f32_leg(C, torch, steps, with_oracle=True):
    """The FP32 precision form on its own workload (384^3, Ra 1e6): FP32
    state and stencil, FP64 norms and Nusselt; plus its per-field error
    against the FP64 form of this library at 128^3 after 100 steps."""
    n, Ra, seed = 384, 1e6, 3
    g = C.Grid.cube(n, C.CAV_F32)
    prm = C.Params(Ra=Ra)
    cav = C.Cavity(g, prm).init(seed, 1e-3)
    cav.step(5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cav.step(steps)
    torch.cuda.synchronize()
    t_run = time.perf_counter() - t0
    C.cavity_timing_read()
    C.cavity_timing_enable(True)
    cav.step(steps)
    torch.cuda.synchronize()
    C.cavity_timing_enable(False)
    kt = C.cavity_timing_read()
    sw_n = sum(kt[k][0] for k in ("sweep", "sweep_norm") if k in kt)
    sw_ms = sum(kt[k][1] for k in ("sweep", "sweep_norm") if k in kt) / sw_n
    ncell = g.ncell
    C.cavity_timing_read()
    C.cavity_timing_enable(True)
    for _ in range(20):
        C.cavity_stream_copy(g, cav.q, cav.q_tmp)
    torch.cuda.synchronize()
    C.cavity_timing_enable(False)
    n_sc, ms_sc = C.cavity_timing_read()["stream_copy"]
    sc_us = 1e3 * ms_sc / n_sc
    out = {"workload": "cavity384_f32_ra1e6", "steps": steps, "value": ncell * steps / t_run,
           "unit": "grid-point updates/s", "ms_per_step": 1e3 * t_run / steps,
           "sweep_avg_us": 1e3 * sw_ms, "sweep_GBs": 40.0 * ncell / (sw_ms * 1e-3) / 1e9,
           "sweep_frac_hbm": 40.0 * ncell / (sw_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "ceiling": {"kernel": "stream_copy_kernel", "avg_launch_us": sc_us,
                       "GBs": 40.0 * ncell / (sc_us * 1e-6) / 1e9, "frac": 40.0 * ncell / (sc_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                       "sweep_over_ceiling_time": 1e3 * sw_ms / sc_us},
           "residual_norms_f64": cav.norms(), "nusselt_f64": cav.nusselt()}
    counted = f32_batch_counter_bytes().get("f32_sweep")
    if counted:
        # HBM bytes by the counters (profiles/) over this run's sweep time
        out["sweep_counter_GBs"] = counted / (sw_ms * 1e-3) / 1e9
        out["sweep_counter_frac"] = out["sweep_counter_GBs"] / HBM_PEAK_GBS
    del cav
    # accuracy: FP32 vs FP64 GPU from the same start, 128^3, 100 steps
    m = 128
    g64, g32 = C.Grid.cube(m), C.Grid.cube(m, C.CAV_F32)
    a = C.Cavity(g64, prm).init(seed, 1e-3)
    b = C.Cavity(g32, prm)
    C.state_view(g32, b.q).copy_(C.state_view(g64, a.q).to(torch.float32))
    a.step(100)
    b.step(100)
    torch.cuda.synchronize()
    A = C.state_view(g64, a.q)[:, 2:-2, 2:-2, 2:-2]
    B = C.state_view(g32, b.q)[:, 2:-2, 2:-2, 2:-2].to(torch.float64)
    err = [float((B[f] - A[f]).abs().max() / A[f].abs().max()) for f in range(5)]
    out["rel_err_vs_f64_gpu_128cubed_100steps"] = dict(zip(("p", "u", "v", "w", "T"), err))
    out["nusselt_128cubed"] = {"f64": a.nusselt(), "f32": b.nusselt()}
    del a, b, A, B
    if with_oracle:
        out.update(f32_vs_oracle(C, torch, n, Ra, seed, steps))
    return out


def f32_vs_oracle(C, torch, n, Ra, seed, steps):
    """The timed FP32 workload from its seeded start, `steps` steps, against
    the FP64 oracle run from the same (FP32-rounded) start on the host cores:
    per-field relative error (max |a - b| / max |b| over the interior).  The
    oracle's stepping loop is timed as the 384^3 FP64 CPU reference."""
    import numpy as np
    import oracle as O
    g = C.Grid.cube(n, C.CAV_F32)
    cav = C.Cavity(g, C.Params(Ra=Ra)).init(seed, 1e-3)
    q0 = np.ascontiguousarray(C.state_view(g, cav.q).cpu().numpy(), dtype=np.float64)
    cav.step(steps)
    got = C.state_view(g, cav.q)[:, 2:-2, 2:-2, 2:-2].cpu().numpy()
    nusselt_gpu = cav.nusselt()
    del cav
    P = O.Problem(n, Ra=Ra)
    t0 = time.perf_counter()
    O.step(P, q0, steps)
    dt = time.perf_counter() - t0
    ref = P.interior(q0)
    err = [float(np.abs(got[f].astype(np.float64) - ref[f]).max() / np.abs(ref[f]).max()) for f in range(5)]
    log("bench: f32 %d^3 x%d vs FP64 oracle: %s (oracle %.1f s)" % (n, steps, err, dt))
    return {"rel_err_vs_f64_oracle_%dcubed_%dsteps" % (n, steps): dict(zip(("p", "u", "v", "w", "T"), err)),
            "nusselt_vs_oracle": {"f32_gpu": nusselt_gpu, "f64_oracle": O.nusselt_hot(P, q0)},
            "tolerance_per_field": 1e-5,
            "oracle_run": {"value": P.ncell * steps / dt, "unit": "grid-point updates/s",
                           "ssspnt_np1": P.ncell * steps / dt * 1e-7, "seconds": dt, "threads": O.threads(),
                           "what": "FP64 oracle, %d^3 Ra %g, %d steps from the rounded start" % (n, Ra, steps)}}


def batch_leg(C, torch, steps, with_oracle=True):
    """The batched form: 96 FP32 cubes of uneven edges and Rayleigh numbers,
    tile shape and k chunk per edge and the block count tuned on the whole
    batch (autotune.tune_batch), `steps` steps replayed from one HIP graph."""
    from paper_2006_02602_amd import autotune
    from paper_2006_02602_amd.configs import batch_workload
    wl = batch_workload()
    b = C.Batch([(C.Grid.cube(e, C.CAV_F32), C.Params(Ra=ra)) for e, ra, _ in wl])
    b.init([s for _, _, s in wl])
    shapes, nb, tb = autotune.tune_batch(b, [e for e, _, _ in wl], C.CAV_F32,
                                         cache_path="/tmp/cavity_autotune.json")
    b.init([s for _, _, s in wl])
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        gr = b.graph(steps, nblocks=nb, stream=st)
        gr.launch(stream=st)
        st.synchronize()
        t0 = time.perf_counter()
        gr.launch(stream=st)
        st.synchronize()
        dt = time.perf_counter() - t0
        gr.destroy()
    norms_ok = all(all(x == x and abs(x) < 1e30 for x in b.norms(m)) for m in range(len(b)))
    acc = batch_vs_oracle(C, torch, b, wl, steps, nb) if with_oracle else None
    counted = f32_batch_counter_bytes().get("batch")
    res = {"workload": "batch96_f32_edges24-96_ra1e3-1e6", "members": len(b), "cells": b.cells,
            "steps": steps, "value": b.cells * steps / dt, "unit": "grid-point updates/s",
            "ms_per_step": 1e3 * dt / steps, "launch": "one persistent kernel per step, %d steps in one HIP graph" % steps,
            "autotuned_tile_and_kc_per_edge": {str(k): {"tile": "%dx%d" % C.batch_tile(C.CAV_F32, v[0]), "kc": v[1]}
                                               for k, v in shapes.items()},
            "autotuned_blocks": nb,
            "block_timings_ms": tb.get("blocks", {}),
            "tuning_trials": len([k for k in tb if k != "blocks"]),
            "bytes_per_step_algorithmic": 40 * b.cells,
            "GBs_algorithmic": 40 * b.cells / (dt / steps) / 1e9, "norms_finite": norms_ok,
            "rel_err_vs_f64_oracle_sampled": acc}
    if counted:
        # HBM bytes per step by the counters (profiles/, taken at that run's
        # tuned shapes) over this run's time per step
        res["counter_GBs"] = counted / (dt / steps) / 1e9
        res["counter_frac"] = res["counter_GBs"] / HBM_PEAK_GBS
    return res


def batch_vs_oracle(C, torch, b, wl, steps, nb):
    """Sampled members (the first of every edge, the lowest and the highest
    Ra) of the batch after `steps` graph-replayed steps from the seeded
    start, against the FP64 oracle from the same (FP32-rounded) start."""
    import numpy as np
    import oracle as O
    b.init([s for _, _, s in wl])
    q0 = {}
    pick = {}
    for m, (e, ra, _) in enumerate(wl):
        pick.setdefault("edge%d" % e, m)
    pick["ra_min"] = min(range(len(wl)), key=lambda m: wl[m][1])
    pick["ra_max"] = max(range(len(wl)), key=lambda m: wl[m][1])
    for m in set(pick.values()):
        q0[m] = np.ascontiguousarray(C.state_view(b.grids[m], b.state(m)).cpu().numpy(), dtype=np.float64)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        gr = b.graph(steps, nblocks=nb, stream=st)
        gr.launch(stream=st)
        st.synchronize()
        gr.destroy()
    out = {}
    for tag, m in sorted(pick.items(), key=lambda kv: kv[1]):
        e, ra, _ = wl[m]
        P = O.Problem(e, Ra=ra)
        ref = q0[m].copy()
        O.step(P, ref, steps)
        got = C.state_view(b.grids[m], b.state(m))[:, 2:-2, 2:-2, 2:-2].cpu().numpy().astype(np.float64)
        want = P.interior(ref)
        err = [float(np.abs(got[f] - want[f]).max() / np.abs(want[f]).max()) for f in range(5)]
        out[tag] = {"member": m, "edge": e, "Ra": ra, "steps": steps,
                    "rel_err": dict(zip(("p", "u", "v", "w", "T"), err))}
    out["max_rel_err"] = max(max(v["rel_err"].values()) for v in out.values())
    out["tolerance_per_field"] = 1e-5
    return out


def overlap_leg(C, torch, grid, prm, splits, widths, steps):
    """Whole steps with the halo exchange: unsplit (cavity_step) against the
    interior/exterior split (cavity_step_overlap) with the exchange on the
    same stream and on a second stream; per split, ms per step."""
    out = []
    comm = torch.cuda.Stream()
    for split in splits:
        h = C.Halo(split, widths)
        cav = C.Cavity(grid, prm, h).init(2)
        row = {"split": "x".join(map(str, split)), "widths": list(widths)}
        for name, fn in (("unsplit", lambda: cav.step(steps)),
                         ("split_one_stream", lambda: cav.step_overlap(steps)),
                         ("split_two_streams", lambda: cav.step_overlap(steps, comm_stream=comm))):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            row[name + "_ms_per_step"] = 1e3 * (time.perf_counter() - t0) / steps
        C.cavity_timing_read()
        C.cavity_timing_enable(True)
        cav.step(steps)
        torch.cuda.synchronize()
        C.cavity_timing_enable(False)
        kt = C.cavity_timing_read()
        # per launch; within a call the sweep of a split along i packs the
        # next exchange (sweep_xpack), so only the first step runs the pack
        row["unsplit_kernels"] = {k: {"launches": n, "avg_us": round(1e3 * ms / n, 2)} for k, (n, ms) in sorted(kt.items())
                                  if k in ("sweep", "sweep_xpack", "sweep_norm", "halo_pack", "halo_unpack")}
        row["unsplit_exchange_us_per_step"] = round(1e3 * sum(kt[k][1] for k in ("halo_pack", "halo_unpack") if k in kt) / steps, 2)
        C.cavity_timing_read()
        C.cavity_timing_enable(True)
        cav.step_overlap(steps, comm_stream=comm)
        torch.cuda.synchronize()
        C.cavity_timing_enable(False)
        kt = C.cavity_timing_read()
        row["split_kernels_us"] = {k: round(1e3 * ms / n, 2) for k, (n, ms) in sorted(kt.items())
                                   if k in ("interior", "interior_norm", "exterior", "exterior_norm", "halo_pack", "halo_unpack")}
        out.append(row)
        del cav
    return out


def adjoint_leg(C, torch):
    """Gradient of the hot-wall Nusselt number (64^3, Ra 1e4, 400 steps,
    checkpoints every 20): forward with checkpoints, then the reverse sweep
    with segment recomputation; plus the reverse step alone at 256^3."""
    from paper_2006_02602_amd.adjoint import NusseltAdjoint
    from paper_2006_02602_amd.configs import ADJOINT as A
    g = A.grid
    th = torch.from_numpy(A.theta()).cuda()
    q0 = torch.zeros(C.cavity_state_elems(g), dtype=torch.float64, device="cuda")
    C.cavity_init(g, C.Params(Ra=A.Ra), A.seed, 1e-3, q0)
    adj = NusseltAdjoint(g, C.Params(), A.steps, A.every, graph=True)
    adj.forward(th, A.Ra, q0)
    torch.cuda.synchronize()
    # the first backward at this Ra runs eagerly and is captured into a graph
    t0 = time.perf_counter()
    adj.backward()
    torch.cuda.synchronize()
    eager_ms = 1e3 * (time.perf_counter() - t0)
    t0 = time.perf_counter()
    J = adj.forward(th, A.Ra, q0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dth, dra, _ = adj.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fwd, bwd = t1 - t0, t2 - t1
    # one reverse step at 64^3 on its own (eager launches, HIP events); the
    # cotangent alternates between two buffers (a step cannot run in place)
    lam64 = (torch.zeros_like(q0), torch.zeros_like(q0))
    C.cavity_nusselt_adjoint(g, C.Params(Ra=A.Ra), lam64[0], None)
    aws64 = torch.empty(C.cavity_adjoint_workspace_bytes(g) // 8, dtype=torch.float64, device="cuda")
    C.cavity_timing_read()
    C.cavity_timing_enable(True)
    for r in range(20):
        C.cavity_adjoint_step(g, C.Params(Ra=A.Ra), q0, lam64[r % 2], lam64[1 - r % 2], aws64, None, None)
    torch.cuda.synchronize()
    C.cavity_timing_enable(False)
    n_rev, rev_ms = C.cavity_timing_read().get("adjoint_step", (0, 0.0))
    del lam64, aws64
    out = {"workload": A.name, "n": A.n, "Ra": A.Ra, "steps": A.steps, "checkpoint_every": A.every,
           "nusselt": J, "dJ_dRa": float(dra.cpu()[0]), "dJ_dtheta_sum": float(dth.sum()),
           "forward_ms": 1e3 * fwd, "gradient_ms": 1e3 * bwd, "gradient_over_forward": bwd / fwd,
           "gradient_is": "replay of the backward pass captured in one HIP graph at this Ra",
           "gradient_first_pass_ms": eager_ms,
           "reverse_step_us": 1e3 * rev_ms / max(n_rev, 1)}
    # the reverse step alone at 256^3 (one GPU's share of the headline grid)
    g2 = C.Grid.cube(256)
    q = torch.zeros(C.cavity_state_elems(g2), dtype=torch.float64, device="cuda")
    C.cavity_init(g2, C.Params(Ra=1e5), 2, 1e-3, q)
    lam = (torch.zeros_like(q), torch.zeros_like(q))
    C.cavity_nusselt_adjoint(g2, C.Params(Ra=1e5), lam[0], None)
    aws = torch.empty(C.cavity_adjoint_workspace_bytes(g2) // 8, dtype=torch.float64, device="cuda")
    for r in range(2):
        C.cavity_adjoint_step(g2, C.Params(Ra=1e5), q, lam[r % 2], lam[1 - r % 2], aws, None, None)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for r in range(reps):
        C.cavity_adjoint_step(g2, C.Params(Ra=1e5), q, lam[r % 2], lam[1 - r % 2], aws, None, None)
    torch.cuda.synchronize()
    us = 1e6 * (time.perf_counter() - t0) / reps
    cells = g2.ncell
    out["reverse_step_256cubed_us"] = us
    out["reverse_step_256cubed_GBs_min_traffic"] = ADJ_MIN_BYTES_PER_CELL * cells / (us * 1e-6) / 1e9
    out["reverse_step_min_bytes_per_cell"] = ADJ_MIN_BYTES_PER_CELL
    counted = adjoint_counter_bytes()
    if counted:
        # HBM bytes per reverse step by the counters (profiles/) over this run's time
        out["reverse_step_256cubed_counter_GBs"] = counted / (us * 1e-6) / 1e9
        out["reverse_step_256cubed_counter_frac"] = out["reverse_step_256cubed_counter_GBs"] / HBM_PEAK_GBS
    del aws, lam, q
    return out


def small_case(C, torch):
    """The 16^3 parity workload (Ra 1e3, 2x2x2 exchange, 100 steps): cache-
    and launch-resident, so only the time per step is reported."""
    from paper_2006_02602_amd.configs import C0
    cav = C.Cavity(C0.grid, C0.params, C0.halo()).init(C0.seed, C0.noise)
    cav.step(10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cav.step(C0.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"workload": "%s_split2x2x2" % C0.name, "steps": C0.steps, "us_per_step": 1e6 * dt / C0.steps,
            "note": "3 launches per step (pack, unpack, sweep); launch-bound, no roofline claim"}


def cpu_model():
    """The host CPU's model string (/proc/cpuinfo), or the platform's."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(wl, budget_s):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    workload (same grid, parameters and halo; fewer steps), plus the 16^3
    parity workload in full (median of 3 runs)."""
    import oracle as O
    from paper_2006_02602_amd.configs import C0
    P = O.Problem(wl.n, Ra=wl.Ra, Pr=0.71, cfl=0.5)
    q = O.init(P, wl.seed, wl.noise)
    halo = (wl.splits[0], wl.widths)
    t0 = time.perf_counter()
    O.step(P, q, 1, halo=halo)
    t1 = time.perf_counter() - t0
    steps = max(1, min(40, int(round(budget_s / max(t1, 1e-3)))))
    t0 = time.perf_counter()
    O.step(P, q, steps, halo=halo)
    dt = time.perf_counter() - t0
    value = P.ncell * steps / dt
    # the small parity case in full: 16^3, Ra 1e3, 100 steps, 2x2x2 exchange
    P0 = O.Problem(C0.n, Ra=C0.Ra)
    runs = []
    for _ in range(3):
        q0 = O.init(P0, C0.seed, C0.noise)
        t0 = time.perf_counter()
        O.step(P0, q0, C0.steps, halo=(C0.splits[0], C0.widths))
        runs.append(time.perf_counter() - t0)
    t_c0 = sorted(runs)[1]
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"value": value, "unit": "grid-point updates/s", "cores": O.threads(),
            "kind": "oracle",
            "sample": "%d^3 Ra %g, %d steps (of %d) with the %s split, whole step timed (%.1f s)"
                      % (wl.n, wl.Ra, steps, wl.steps, "x".join(map(str, wl.splits[0])), dt),
            "ssspnt_np1": value * 1e-7,
            "host": {"cpu_model": cpu_model(), "nproc": usable, "os_cpu_count": os.cpu_count(),
                     "omp_threads": O.threads()},
            "small_case_16cubed_100steps": {"seconds_median_of_3": t_c0, "runs_s": runs,
                                            "value": P0.ncell * C0.steps / t_c0, "unit": "grid-point updates/s"}}


def counter_rates(kernel_hash, avg_us):
    """Counter-based HBM rate of the sweep: the calibrated FETCH_SIZE +
    WRITE_SIZE bytes of one launch (rocprofv3, committed summary tied to the
    sweep source hash) over the launch's average duration."""
    traffic = counter_traffic(kernel_hash)
    if traffic is None:
        return None, None
    gbs = traffic / (avg_us * 1e-6) / 1e9
    return traffic, {"GBs": gbs, "frac": gbs / HBM_PEAK_GBS, "bytes_per_launch": traffic,
                     "time_source": "HIP events around each sweep launch in this run (same stream)",
                     "counters": "profiles/sweep_cavity256_f64_counters.md"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="cavity256_f64_ra1e5")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--no-halo-bench", action="store_true")
    ap.add_argument("--no-f32", action="store_true", help="skip the FP32 precision-form leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-form leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the discrete-adjoint leg")
    ap.add_argument("--no-overlap", action="store_true", help="skip the interior/exterior split leg")
    ap.add_argument("--legs", default=None,
                    help="comma list of extra legs to run (halo,f32,batch,adjoint,overlap; 'none' for the "
                         "headline only); overrides the --no-* flags")
    ap.add_argument("--no-oracle", action="store_true",
                    help="skip the FP32 and batch legs' comparisons with the FP64 oracle (about 45 s of host time)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--halo-reps", type=int, default=10, help="pack/unpack pairs per halo row and mode")
    ap.add_argument("--settle", type=float, default=1.0,
                    help="seconds of continuous stepping before the warm-up steps (clock ramp-up)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.legs is not None:
        want = set(x.strip() for x in args.legs.split(",") if x.strip())
        unknown = want - {"none", "halo", "f32", "batch", "adjoint", "overlap"}
        if unknown:
            ap.error("unknown legs: %s" % ",".join(sorted(unknown)))
        args.no_halo_bench = "halo" not in want
        args.no_f32 = "f32" not in want
        args.no_batch = "batch" not in want
        args.no_adjoint = "adjoint" not in want
        args.no_overlap = "overlap" not in want

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU's share of the cavity; it does not run on %d GPUs "
              "(there is no multi-GPU path in this library)" % max(args.gpus, int(os.environ.get("WORLD_SIZE", "1"))),
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2006_02602_amd as C
    from paper_2006_02602_amd.configs import WORKLOADS

    wl = WORKLOADS[args.workload]
    K = args.steps if args.steps is not None else wl.steps
    W = args.warmup
    torch.cuda.set_device(0)
    grid, prm, halo = wl.grid, wl.params, wl.halo()
    log("bench: %s, %d warmup + %d timed steps, halo %s widths %s" % (wl.name, W, K, halo.split, halo.width))
    cav = C.Cavity(grid, prm, halo).init(wl.seed, wl.noise)
    torch.cuda.synchronize()

    if args.calib_copy:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # Clock settle: the GPU's clocks ramp up under sustained load, and a few
    # milliseconds of work (5 warm-up steps are about 2 ms) leave the sweep
    # ~7% slower than in steady state.  Step continuously for `settle`
    # seconds first (reported below), then the W warm-up steps.
    t0 = time.perf_counter()
    settle_steps = 0
    while time.perf_counter() - t0 < args.settle:
        cav.step(10)
        torch.cuda.synchronize()
        settle_steps += 10
    settle_s = time.perf_counter() - t0
    if W:
        cav.step(W)
    torch.cuda.synchronize()

    # timed region: K whole steps
    t0 = time.perf_counter()
    cav.step(K)
    torch.cuda.synchronize()
    t_run = time.perf_counter() - t0
    norms = cav.norms()
    log("bench: %.3f ms/step, norms %s" % (1e3 * t_run / K, norms))

    # the same K steps again with HIP events around every launch, on the
    # stream each kernel is launched on
    C.cavity_timing_read()
    C.cavity_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cav.step(K)
    torch.cuda.synchronize()
    t_ev = time.perf_counter() - t0
    C.cavity_timing_enable(False)
    kt = C.cavity_timing_read()
    sw_keys = ("sweep", "sweep_xpack", "sweep_norm")
    sw_n = sum(kt[k][0] for k in sw_keys if k in kt)
    sw_ms = sum(kt[k][1] for k in sw_keys if k in kt) / sw_n
    ncell = grid.ncell
    achieved = SWEEP_BYTES_PER_CELL * ncell / (sw_ms * 1e-3) / 1e9
    kh = sweep_source_hash()
    traffic, counter = counter_rates(kh, 1e3 * sw_ms)
    # the sweep's memory streams without its work (same tiles, order, chunks
    # and prefetch depth): the ceiling of its access pattern on this device
    C.cavity_timing_read()
    C.cavity_timing_enable(True)
    for _ in range(K):
        C.cavity_stream_copy(grid, cav.q, cav.q_tmp)
    torch.cuda.synchronize()
    C.cavity_timing_enable(False)
    n_sc, ms_sc = C.cavity_timing_read()["stream_copy"]
    sc_us = 1e3 * ms_sc / n_sc
    ceiling = {"kernel": "stream_copy_kernel", "what": "the sweep's 5 reads + 5 non-temporal writes per interior cell, "
                                                      "same tiles, block order, k chunks and prefetch depth, no work",
               "avg_launch_us": sc_us, "GBs": SWEEP_BYTES_PER_CELL * grid.ncell / (sc_us * 1e-6) / 1e9,
               "frac": SWEEP_BYTES_PER_CELL * grid.ncell / (sc_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
               "sweep_over_ceiling_time": 1e3 * sw_ms / sc_us}
    # the same K steps once more without events: how much of the timed pass
    # is the device settling after the short warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cav.step(K)
    torch.cuda.synchronize()
    t_again = time.perf_counter() - t0
    breakdown = {k: {"launches": n, "avg_us": round(1e3 * ms / n, 2)} for k, (n, ms) in sorted(kt.items())}
    log("bench: sweep %.1f us -> %.0f GB/s algorithmic" % (1e3 * sw_ms, achieved))

    small = small_case(C, torch)
    log("bench: small case", small)

    halo_res = None
    if not args.no_halo_bench:
        splits = wl.splits
        from paper_2006_02602_amd.configs import CONFIG_WIDTHS, PAPER_WIDTHS
        halo_res = halo_bench(C, torch, grid, cav, splits, (CONFIG_WIDTHS, PAPER_WIDTHS), reps=args.halo_reps)
        for r in halo_res:
            log("bench: halo", r)

    f32 = None
    if not args.no_f32:
        log("bench: FP32 form (384^3) ...")
        f32 = f32_leg(C, torch, 100, with_oracle=not args.no_oracle)
        log("bench: f32", f32)

    batch = None
    if not args.no_batch:
        log("bench: batched form (96 cavities) ...")
        batch = batch_leg(C, torch, 100, with_oracle=not args.no_oracle)
        log("bench: batch", batch)

    ovl = None
    if not args.no_overlap:
        log("bench: interior/exterior split ...")
        ovl = overlap_leg(C, torch, grid, prm, wl.splits, wl.widths, 20)
        for r in ovl:
            log("bench: overlap", r)

    adj = None
    if not args.no_adjoint:
        log("bench: discrete adjoint (64^3, 400 steps) ...")
        adj = adjoint_leg(C, torch)
        log("bench: adjoint", adj)

    value = ncell * K / t_run
    line = {
        "metric": "grid-point updates/s + % HBM peak (stencil, pack/unpack); FP32 & batched vs FP64",
        "value": value,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * t_run / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded SplitMix64 noise on rest state, T linear in x)",
        "config": {"workload": "%s_split%s" % (wl.name, "x".join(map(str, halo.split))), "n": wl.n,
                   "Ra": wl.Ra, "Pr": 0.71, "cfl": 0.5, "halo_split": list(halo.split),
                   "halo_widths_p_u_v_w_T": list(halo.width), "parallelism": "single GPU"},
        "ssspnt": value * 1e-7,
        "paper_context": {"ssspnt_single_p100_256cubed": PAPER_SSSPNT_P100,
                          "note": "P100, OpenACC Fortran, no halo in that row; context only"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "sweep_kernel", "bytes_per_launch": SWEEP_BYTES_PER_CELL * ncell,
                     "achieved_is": "algorithmic bytes (80 B per interior cell) / average launch time",
                     "avg_launch_us": 1e3 * sw_ms,
                     "time_source": "HIP events around each sweep launch in this run (same stream)",
                     "counter": counter, "sweep_source_hash": kh,
                     "ceiling": ceiling},
        "breakdown_us_per_launch": breakdown,
        "settle": {"seconds": settle_s, "steps": settle_steps,
                   "why": "untimed continuous steps before the warm-up so that the timed steps run at steady clocks"},
        "ms_per_step_with_events": 1e3 * t_ev / K,
        "ms_per_step_second_pass": 1e3 * t_again / K,
        "residual_norms": norms,
    }
    line["small_case"] = small
    if halo_res is not None:
        line["halo"] = halo_res
    if f32 is not None:
        # updates/s of the FP32 sweep-only step at 384^3 against the FP64
        # sweep rate of the headline run (both exclude the halo exchange)
        f64_sweep_rate = ncell / (sw_ms * 1e-3)
        f32_sweep_rate = f32["value"]
        f32["f32_over_f64_sweep_rate"] = f32_sweep_rate / f64_sweep_rate
        line["f32"] = f32
    if batch is not None:
        batch["batch_over_f64_sweep_rate"] = batch["value"] / (ncell / (sw_ms * 1e-3))
        if f32 is not None:
            batch["batch_over_f32_single_rate"] = batch["value"] / f32["value"]
        line["batch"] = batch
    if ovl is not None:
        line["overlap"] = ovl
    if adj is not None:
        adj["reverse_over_forward_step_256cubed"] = adj["reverse_step_256cubed_us"] / (1e3 * sw_ms)
        line["adjoint"] = adj
    if not args.no_cpu:
        log("bench: CPU baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget)
        if f32 is not None and "oracle_run" in f32:
            line["cpu_baseline"]["f64_384cubed_100steps"] = f32["oracle_run"]
        log("bench: CPU baseline", line["cpu_baseline"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
