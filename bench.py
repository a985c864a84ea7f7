#!/usr/bin/env python3
"""Benchmark of the embedding-ERI build (Alg. 1) on one MI355X.

One step = one pass of the whole path on the resident inputs: the bath SVD and
C^k, the one-body transforms of h and gamma with E1, then dmet_transform_eri
(the k-AO to k-EO transform of the GDF 3-index tensor for every fitting
momentum q and the packed contraction, for every spin block: alpha-alpha,
beta-beta, alpha-beta).  The ERI build alone is reported as eri_build_ms.

Prints ONE JSON line.  ``value`` is the useful throughput W / t in TFLOP/s,
W = W_T + W_C with W_T = 8 N_k^2 naux (nao^2 neo + nao neo^2) per spin (all
(q, k) pairs of Alg. 1, 8 real flops per complex MAC) and W_C the minimal real
contraction count N_k naux npair (npair + 1) per same-spin block plus
2 N_k naux npair^2 for the alpha-beta block.
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

import numpy as np  # noqa: E402

METRIC = "embedding-ERI build s + TFLOP/s, split-BF16/FP32 vs FP64 at ≤1e-6 max err"
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "bf16x6": 2500.0, "bf16x6_i8": 2500.0}   # dense MFMA TFLOP/s
PEAK_I8 = 5000.0   # dense int8 MFMA TOP/s (MI355X spec): the peak of the int8 contraction kernels
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3", "bf16x6": "bf16x6", "bf16x6_i8": "bf16x6+int8x3"}


def _nk3(kmesh):
    return int(kmesh[0]) * int(kmesh[1]) * int(kmesh[2])


def kernel_peak(prec, name):
    """Dense MFMA peak of the dtype the named kernel multiplies in."""
    return PEAK_I8 if name.endswith("_i8") else PEAK[prec]


def work_counts(wl):
    nk, nao, naux, neo, ns = wl.nk, wl.nao, wl.naux, wl.neo, wl.nspin
    npair = neo * (neo + 1) // 2
    wt = 8.0 * nk * nk * naux * (nao * nao * neo + nao * neo * neo) * ns
    wc = nk * naux * npair * (npair + 1.0) * ns + (2.0 * nk * naux * npair * npair if ns == 2 else 0.0)
    return wt, wc


def kernel_flops(wl, name):
    """Algorithmic flops of ONE launch of the named kernel: stage 1 of Alg. 1 for one q over all k
    and both spins (8 real flops per complex MAC), stage 2 for one q and spin over the i >= j half, and the
    packed contraction of one spin block (two flops per MAC over IJ >= KL, or the full alpha-beta
    square)."""
    nk, nao, naux, neo = wl.nk, wl.nao, wl.naux, wl.neo
    npair = neo * (neo + 1) // 2
    if name.startswith("xform1"):
        return 8.0 * nk * naux * nao * nao * neo * wl.nspin
    if name.startswith("xform2"):
        return 8.0 * nk * naux * nao * neo * (neo + 1) / 2
    if name.startswith("contract_s8"):
        return nk * naux * npair * (npair + 1.0)
    if name.startswith("contract_s4"):
        return 2.0 * nk * naux * npair * float(npair)
    return None


MFMA_PRODUCTS = {"fp64": 1, "fp32": 1, "bf16x3": 3, "bf16x6": 6, "bf16x6_i8": 6}   # executed per algorithmic product


def traffic_bytes(kernel, workload):
    """HBM bytes per launch of `kernel` from profiles/traffic.json, if the
    counters were taken on this workload with the current kernel source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        tr = json.load(open(path))
        e = tr[kernel]
        sha = hashlib.sha1(open(os.path.join(ROOT, e["source"]), "rb").read()).hexdigest()
    except (OSError, KeyError, ValueError):
        return None
    if e.get("workload") != workload or e.get("source_sha1") != sha:
        return None
    return e["fetch_bytes"] + e["write_bytes"]


def coulomb_exchange_energies(out, g_eo, chunk=1 << 27):
    """E_J = 1/2 sum (ij|kl) g_ji g_lk and E_K = 1/2 sum (ij|kl) g_jk g_li per
    spin block, from the packed outputs of one form (device tensors; g_eo
    [nspin][neo][neo] float64, symmetric).  The s8 block is summed over its
    stored triangle with the multiplicity of each element's symmetry images;
    the alpha-beta block (s4) has a Coulomb term only.  Measurement helper of
    the benchmark, not part of the library."""
    import torch
    neo = g_eo.shape[-1]
    npair = neo * (neo + 1) // 2
    dev = g_eo.device
    tri_i, tri_j = torch.tril_indices(neo, neo, device=dev)

    def pair_weight(g):        # g~[IJ] = g_ij (2 - delta_ij): sum over (i,j) and (j,i)
        return g[tri_i, tri_j] * torch.where(tri_i == tri_j, 1.0, 2.0).to(g.dtype)

    def k_weight(ga, gb, i, j, k, l):
        # sum over the index orders of the two pairs of gb_{bc} ga_{da}, each
        # distinct ordering once
        t = ga[l, i] * gb[j, k]
        t = t + torch.where(i != j, ga[l, j] * gb[i, k], torch.zeros_like(t))
        t = t + torch.where(k != l, ga[k, i] * gb[j, l], torch.zeros_like(t))
        t = t + torch.where((i != j) & (k != l), ga[k, j] * gb[i, l], torch.zeros_like(t))
        return t

    res = {}
    for key, e in out.items():
        sa, sb = {"aa": (0, 0), "bb": (1, 1), "ab": (0, 1)}[key]
        ga, gb = g_eo[sa], g_eo[sb]
        wa, wb = pair_weight(ga), pair_weight(gb)
        ej = torch.zeros((), dtype=torch.float64, device=dev)
        ek = torch.zeros((), dtype=torch.float64, device=dev)
        flat = e.reshape(-1)
        for s0 in range(0, flat.numel(), chunk):
            idx = torch.arange(s0, min(flat.numel(), s0 + chunk), device=dev, dtype=torch.int64)
            v = flat[s0:s0 + idx.numel()]
            if key == "ab":
                IJ, KL = idx // npair, idx % npair
                ej += (v * wa[IJ] * wb[KL]).sum()
                continue
            IJ = ((torch.sqrt(8.0 * idx.double() + 1.0) - 1.0) / 2.0).floor().long()
            IJ = IJ - (IJ * (IJ + 1) // 2 > idx).long()
            IJ = IJ + ((IJ + 1) * (IJ + 2) // 2 <= idx).long()
            KL = idx - IJ * (IJ + 1) // 2
            mult = torch.where(IJ == KL, 1.0, 2.0).double()
            ej += (v * mult * wa[IJ] * wa[KL]).sum()
            i, j, k, l = tri_i[IJ], tri_j[IJ], tri_i[KL], tri_j[KL]
            ek += (v * mult * k_weight(ga, ga, i, j, k, l)).sum()
        res[key] = {"E_J": 0.5 * float(ej)} if key == "ab" else {"E_J": 0.5 * float(ej), "E_K": 0.5 * float(ek)}
    return res


def host_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    mem = 0
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                mem = int(line.split()[1]) // (1024 * 1024)
    except OSError:
        pass
    return model, mem


def cpu_baseline(wl, lat, lm, n_l, n_rows, imp_idx=None, val_idx=None, w_flop=None, one_thread=False):
    """Time the FP64 oracle on a bounded sample of the same workload, phase by
    phase, and extrapolate its time for the whole workload:

    * bath (Eqs. bath R SVD, C loemb R/k) and the one-body transforms of h and
      gamma: timed in full;
    * transform (the embedded 3-index of Alg. 1): q = 0 for the first n_l
      fitting functions over every k, scaled by N_k q-points, naux / n_l and
      the spins;
    * contraction: that block's contribution to n_rows output pair rows (the
      oracle forms the full square over all neo^2 pairs in complex
      arithmetic), scaled by neo^2 / n_rows, naux / n_l, N_k and the spin
      blocks (aa, or aa, bb and ab).

    ``value`` = W / t_oracle(extrapolated) on the same useful-work convention W
    as the GPU's value; the sample's own executed rate is reported too.  With
    one_thread (the small workloads) the same sample is timed again with the
    BLAS held to one thread."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import kspace as ok
    n = wl.neo
    nblocks = 3 if wl.nspin == 2 else 1

    def sample():
        t0 = time.perf_counter()
        bath = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao, imp_idx=imp_idx, val_idx=val_idx)
        t1 = time.perf_counter()
        ok.transform_1e(bath["c_k"], lat.h_k)
        ok.transform_1e(bath["c_k"], lat.dm_k)
        t2 = time.perf_counter()
        ck = bath["c_k"][0]
        sub = lm[:, :, :n_l]
        t3 = time.perf_counter()
        x = ok.alg1_embedded_3index(sub, ck, wl.kmesh, 0)
        t4 = time.perf_counter()
        xm = x.reshape(n_l, -1)
        e = (xm[:, :n_rows].conj().T @ xm) / wl.nk
        t5 = time.perf_counter()
        del e
        t_tr = (t4 - t3) * wl.nk * (wl.naux / n_l) * wl.nspin
        t_co = (t5 - t4) * (n * n / n_rows) * (wl.naux / n_l) * wl.nk * nblocks
        return t0, t1, t2, t3, t4, t5, t_tr, t_co

    t0, t1, t2, t3, t4, t5, t_tr, t_co = sample()
    t_all = (t1 - t0) + (t2 - t1) + t_tr + t_co
    flops = 8.0 * wl.nk * n_l * (wl.nao * wl.nao * n + wl.nao * n * n) + 8.0 * n_l * n_rows * n * n
    info = threadpool_info()
    threads = max([p.get("num_threads", 1) for p in info] or [1])
    blas = ", ".join(sorted({f"{p.get('internal_api')} {p.get('version')}" for p in info if p.get("user_api") == "blas"}))
    out = {"unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
           "sample": f"oracle (numpy FP64, {blas}, {threads} threads): bath and one-body timed in full; Alg. 1 "
                     f"transform of q=0 for {n_l} of {wl.naux} fitting functions over all {wl.nk} k, and that "
                     f"block's contraction for {n_rows} of {n * n} pair rows (spin alpha); whole-workload time "
                     f"extrapolated from these ({t_all:.0f} s)",
           "seconds": t5 - t0, "extrapolated_s": round(t_all, 1),
           "phases_s": {"bath": round(t1 - t0, 3), "onebody": round(t2 - t1, 3),
                        "transform_extrapolated": round(t_tr, 1), "contraction_extrapolated": round(t_co, 1)},
           "sample_rate_TFLOPs": round(flops / ((t5 - t3)) / 1e12, 4), "blas": blas}
    out["value"] = (w_flop / t_all / 1e12) if w_flop else out["sample_rate_TFLOPs"]
    if one_thread:
        with threadpool_limits(limits=1):
            u0, u1, u2, u3, u4, u5, u_tr, u_co = sample()
        u_all = (u1 - u0) + (u2 - u1) + u_tr + u_co
        out["one_thread"] = {"seconds": round(u5 - u0, 3), "extrapolated_s": round(u_all, 2),
                             "phases_s": {"bath": round(u1 - u0, 3), "onebody": round(u2 - u1, 3),
                                          "transform_extrapolated": round(u_tr, 2),
                                          "contraction_extrapolated": round(u_co, 2)}}
    return out


def hbm_copy_rate(dev, gib=2.0, reps=5):
    """HBM rate of a plain device-to-device copy measured on this GPU: bytes
    read plus bytes written per second (TB/s), for comparison with the 8 TB/s
    spec that the rooflines use."""
    import torch
    n = int(gib * (1 << 30)) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        b.copy_(a)
    e1.record(st)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3
    del a, b
    return round(2.0 * 4 * n * reps / t / 1e12, 3)


def run_batched(args, dev):
    """Config-5-like batch: 64 fragments, neo ~ U{20..200}, supercell impurities,
    2x2x2 / 3x3x3 meshes, nao 52, naux 400, complex64 3-index.  Times one batched
    submission (graph replay, autotuned contraction tile) against the loop of
    single-fragment calls, for each requested form."""
    import torch
    import synth
    from paper_1909_08596_amd import dmet

    t0 = time.perf_counter()
    lats = {}
    for name, wl in synth.BATCH_LATTICES.items():
        lat = synth.make_lattice(wl)
        lm = synth.three_index(wl).astype(np.complex64)
        lats[name] = (wl, lat, torch.from_numpy(lm).to(dev), torch.from_numpy(lat.dm_k).to(dev))
        del lm
    specs_in = synth.batched_fragments(args.nfrag)
    print(f"[bench] batched inputs in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    frags, wsum = [], 0.0
    t0 = time.perf_counter()
    for fs in specs_in:
        wl, lat, lm_d, dm_d = lats[fs["lattice"]]
        ck, sv, neo = dmet.dmet_build_bath(wl.kmesh, wl.nao, dm_d, imp_idx=fs["imp_idx"], val_idx=fs["val_idx"])
        ck = ck[0, :, :, : neo[0]].contiguous()
        frags.append({"kmesh": wl.kmesh, "nao": wl.nao, "naux": wl.naux, "lmunu": lm_d, "c_k": ck})
        n = neo[0]
        npair = n * (n + 1) // 2
        wsum += 8.0 * wl.nk * wl.nk * wl.naux * (wl.nao * wl.nao * n + wl.nao * n * n)
        wsum += wl.nk * wl.naux * npair * (npair + 1.0)
    torch.cuda.synchronize()
    t_bath = time.perf_counter() - t0
    neos = [f["c_k"].shape[-1] for f in frags]
    forms = [args.precision] + [p for p in args.compare.split(",") if p and p != args.precision and p != "fp64"]
    out = {}
    # plain FP64 path over the same batch (the per-fragment FP64 kernels): the
    # reference for every form's speed-up and max error
    ws = torch.empty(dmet.dmet_transform_eri_batched_workspace(frags, "fp64"), dtype=torch.uint8, device=dev)
    dmet.dmet_transform_eri_batched(frags, "fp64", workspace=ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        dmet.dmet_transform_eri_batched(frags, "fp64", workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    ms_64 = e0.elapsed_time(e1) / args.steps
    ref64 = [f.pop("eri") for f in frags]
    del ws
    out["fp64"] = {"ms_batched": round(ms_64, 3), "TFLOP/s": round(wsum / (ms_64 * 1e-3) / 1e12, 3)}
    print(f"[bench] batched fp64: {ms_64:.2f} ms", file=sys.stderr, flush=True)
    for prec in forms:
        ws = torch.empty(dmet.dmet_transform_eri_batched_workspace(frags, prec), dtype=torch.uint8, device=dev)
        ws_b = ws
        for _ in range(max(1, args.warmup)):
            dmet.dmet_transform_eri_batched(frags, prec, graph=True, autotune=True, workspace=ws)
        torch.cuda.synchronize()
        dmet.dmet_profile_reset()
        dmet.dmet_profile_enable(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            dmet.dmet_transform_eri_batched(frags, prec, graph=True, autotune=True, workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        dmet.dmet_profile_enable(False)
        ms_b = e0.elapsed_time(e1) / args.steps
        err64 = max(float((f["eri"] - r).abs().max()) for f, r in zip(frags, ref64))
        ref = [f["eri"].clone() for f in frags]
        # loop of single-fragment calls, same precision
        loop_ws = torch.empty(max(dmet.dmet_transform_eri_workspace(f["kmesh"], f["nao"], f["naux"], 1,
                                                                    f["c_k"].shape[-1], prec, f["lmunu"].dtype)
                                  for f in frags), dtype=torch.uint8, device=dev)
        outs = [{"aa": f["eri"]} for f in frags]
        for f, o in zip(frags, outs):
            dmet.dmet_transform_eri(f["kmesh"], f["nao"], f["naux"], f["lmunu"], f["c_k"][None], prec,
                                    workspace=loop_ws, out=o)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            for f, o in zip(frags, outs):
                dmet.dmet_transform_eri(f["kmesh"], f["nao"], f["naux"], f["lmunu"], f["c_k"][None], prec,
                                        workspace=loop_ws, out=o)
        e1.record()
        torch.cuda.synchronize()
        ms_l = e0.elapsed_time(e1) / args.steps
        same = all(torch.equal(a, o["aa"]) for a, o in zip(ref, outs))
        out[prec] = {"ms_batched": round(ms_b, 3), "ms_loop": round(ms_l, 3),
                     "speedup_batched_vs_loop": round(ms_l / ms_b, 3),
                     "TFLOP/s": round(wsum / (ms_b * 1e-3) / 1e12, 3), "batched_equals_loop": bool(same),
                     "speedup_vs_fp64": round(ms_64 / ms_b, 3), "max_abs_err_vs_fp64": err64}
        # one eager submission with the library's phase timing (a graph replay is one span), and the
        # contraction phase against its MFMA peak: algorithmic flops summed over the fragments
        dmet.dmet_profile_reset()
        dmet.dmet_profile_enable(True)
        dmet.dmet_transform_eri_batched(frags, prec, graph=False, autotune=True, workspace=ws_b)
        torch.cuda.synchronize()
        dmet.dmet_profile_enable(False)
        prof = dmet.dmet_profile_report()
        out[prec]["phases_ms_eager"] = {k: round(v[1], 3) for k, v in prof.items()}
        cname = [k for k in prof if k.startswith("batch_contract")]
        if cname:
            t_c = prof[cname[0]][1]
            w_c = sum(_nk3(f["kmesh"]) * f["naux"] * (n * (n + 1) // 2) * (n * (n + 1) // 2 + 1.0)
                      for f in frags for n in [f["c_k"].shape[-1]])
            peak = PEAK_I8 if prec == "bf16x6_i8" else PEAK[prec]
            ach = w_c / (t_c * 1e-3) / 1e12
            out[prec]["contraction_roofline"] = {
                "bound": "mfma", "kernel": cname[0], "ms": round(t_c, 3), "flop": w_c, "achieved": round(ach, 3),
                "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 4),
                "mfma_util": round(ach * MFMA_PRODUCTS[prec] / peak, 4), "traffic": None}
        print(f"[bench] batched {prec}: {ms_b:.2f} ms vs loop {ms_l:.2f} ms; equal={same}; "
              f"{ms_64 / ms_b:.2f}x fp64, max err {err64:.2e}", file=sys.stderr, flush=True)
        del ws, ws_b, loop_ws
    head = out[args.precision]
    line = {
        "metric": METRIC, "value": head["TFLOP/s"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_batched"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": f"batched: {len(frags)} fragments, neo {min(neos)}-{max(neos)} (mean "
                               f"{sum(neos) / len(neos):.0f}), k-meshes 2x2x2 / 3x3x3, nao 52, naux 400, "
                               f"supercell impurities, 3-index complex64", "W_flop": wsum},
        "forms": out, "bath_s_all_fragments": round(t_bath, 3),
    }
    if "contraction_roofline" in head:
        line["roofline"] = head["contraction_roofline"]
    print(json.dumps(line), flush=True)


def run_fftdf(args, dev):
    """Plane-wave (FFTDF) embedding ERIs, App. B / Alg. 2: Gaussian AOs on a 16^3
    grid of a 5.1 bohr cubic cell, 2x2x2 mesh, 26 AOs, 52 EOs; FP64, or with
    --precision bf16x6 / bf16x3 the split-bf16 transform and contraction (the
    grid DFT in FP64), then also compared with FP64 on every element."""
    import torch
    import synth
    from paper_1909_08596_amd import dmet
    wl, g = synth.FFT_CONFIGS[args.config]
    print(f"[bench] generating {wl.name} plane-wave inputs", file=sys.stderr, flush=True)
    lat = synth.make_lattice(wl)
    rho = synth.fftdf_pair_density(wl, g)
    rho_d = torch.from_numpy(rho).to(dev)
    dm_d = torch.from_numpy(lat.dm_k).to(dev)
    ck, _, _ = dmet.dmet_build_bath(wl.kmesh, wl.nao, dm_d)
    prec = args.precision if args.precision in ("fp64", "bf16x6", "bf16x3") else "fp64"
    ws = torch.empty(1, dtype=torch.uint8, device=dev)
    err64 = None
    if prec != "fp64":
        ref = dmet.dmet_transform_eri_fftdf(wl.kmesh, wl.nao, g.n, g.cell, rho_d, ck)["aa"]
        got = dmet.dmet_transform_eri_fftdf(wl.kmesh, wl.nao, g.n, g.cell, rho_d, ck, precision=prec)["aa"]
        err64 = float((got - ref).abs().max())
        del ref, got
    out = dmet.dmet_transform_eri_fftdf(wl.kmesh, wl.nao, g.n, g.cell, rho_d, ck, precision=prec)
    for _ in range(max(0, args.warmup - 1)):
        out = dmet.dmet_transform_eri_fftdf(wl.kmesh, wl.nao, g.n, g.cell, rho_d, ck, precision=prec)
    torch.cuda.synchronize()
    dmet.dmet_profile_reset()
    dmet.dmet_profile_enable(True)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(args.steps):
        out = dmet.dmet_transform_eri_fftdf(wl.kmesh, wl.nao, g.n, g.cell, rho_d, ck, precision=prec)
    e1.record(st)
    torch.cuda.synchronize()
    dmet.dmet_profile_enable(False)
    prof = dmet.dmet_profile_report()
    ms = e0.elapsed_time(e1) / args.steps
    del ws, out
    nk, nr, nao, neo = wl.nk, g.nr, wl.nao, wl.neo
    npair = neo * (neo + 1) // 2
    wt = 8.0 * nk * nk * nr * (nao * nao * neo + nao * neo * neo)
    wfft = nk * npair * 5.0 * nr * math.log2(nr)
    wc = nk * nr * npair * (npair + 1.0)
    dname, (dn, dms) = max(prof.items(), key=lambda kv: kv[1][1])
    avg = dms / dn
    # per launch (group): stage 1 / stage 2 of one q over all k, the contraction of one spin block, and the
    # grid DFT of one q block (three axis passes, each output an n_d-point complex sum: 8 flop per term)
    kflops = {"xform1": 8.0 * nk * nr * nao * nao * neo, "xform2": 8.0 * nk * nr * nao * neo * (neo + 1) / 2,
              "contract_s8": wc, "fftdf": 8.0 * npair * nr * sum(g.n)}
    kf = kflops.get(dname.rsplit("_", 1)[0])
    peak = kernel_peak(prec, dname) if kf is not None and not dname.endswith("f64") else PEAK["fp64"]
    bound = "mfma"
    if dname == "fftdf_dft":
        bound, peak = "alu", PEAK["fp64"]   # FP64 vector arithmetic: 78.6 TFLOP/s on MI355X
    line = {
        "metric": METRIC, "value": round((wt + wfft + wc) / (ms * 1e-3) / 1e12, 4), "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[prec], "data": "synthetic",
        "config": {"workload": f"{wl.name}: plane-wave density fitting (App. B), k-mesh {'x'.join(map(str, wl.kmesh))}, "
                               f"grid {'x'.join(map(str, g.n))} in a {g.cell[0]} bohr cell, nao {nao}, neo {neo}, "
                               f"Gaussian AOs, pair density complex128",
                   "precision": prec, "W_flop": wt + wfft + wc, "W_T": wt, "W_FFT": wfft, "W_C": wc},
        "roofline": {"bound": bound, "kernel": dname, "achieved": None if kf is None else round(kf / (avg * 1e-3) / 1e12, 3),
                     "peak": peak, "unit": "TFLOP/s",
                     "frac": None if kf is None else round(kf / (avg * 1e-3) / 1e12 / peak, 4),
                     "traffic": None, "launch_ms": round(avg, 4), "flop_per_launch": kf},
        "kernels_ms_per_step": {k: round(v[1] / args.steps, 3) for k, v in prof.items()},
    }
    if err64 is not None:
        line["max_abs_err_vs_fp64"] = err64
    if not args.no_cpu_baseline:
        from oracle import kspace as ok
        from threadpoolctl import threadpool_info
        bath = ok.build_bath(lat.dm_k, wl.kmesh, wl.nao)
        t0 = time.perf_counter()
        # one q of Alg. 2 (of N_k): transform, FFT, kernel, inverse FFT, contraction
        e, _ = ok.alg2_eri(rho[:1, :1], bath["c_k"][0][:1], (1, 1, 1), g.n, g.cell)
        t1 = time.perf_counter()
        fl = (8.0 * nr * (nao * nao * neo + nao * neo * neo) + 2.0 * neo * neo * 5.0 * nr * math.log2(nr)
              + 8.0 * nr * neo ** 4)
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
        line["cpu_baseline"] = {"value": fl / (t1 - t0) / 1e12, "unit": "TFLOP/s", "cores": int(threads),
                                "kind": "oracle",
                                "sample": f"oracle Alg. 2 for one (q, k) block of {nk * nk}: transform, FFT, kernel, "
                                          f"inverse FFT and grid contraction of {neo * neo} EO pairs; "
                                          f"{fl:.3e} flop in {t1 - t0:.2f} s", "seconds": t1 - t0}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="nio",
                    help="synthetic workload (tiny, hbn, si, nio, bn33 = the paper's timed BN 3x3x1 shape, batched, "
                         "fft_si = plane-wave density fitting)")
    ap.add_argument("--precision", default="bf16x6_i8", choices=["fp64", "fp32", "bf16x3", "bf16x6", "bf16x6_i8"],
                    help="form whose throughput is `value` (bf16x6_i8: the fastest form within 1e-6 Ha)")
    ap.add_argument("--compare", default="fp64,fp32,bf16x6,bf16x3",
                    help="comma list of other precisions to time and compare against fp64 ('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-l", type=int, default=0, help="fitting functions in the CPU sample (0: naux/2)")
    ap.add_argument("--cpu-sample-rows", type=int, default=16384)
    ap.add_argument("--nfrag", type=int, default=64, help="fragments of the batched workload")
    ap.add_argument("--copy-calib-gib", type=float, default=0.0,
                    help="only run a plain device-to-device copy of this many GiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_calib_gib > 0:
        import torch
        n = int(args.copy_calib_gib * (1 << 30)) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n}))
        return

    import torch
    import synth
    from paper_1909_08596_amd import dmet

    dev = torch.device("cuda:0")
    dmet.load()
    if args.config == "batched":
        run_batched(args, dev)
        return
    if args.config in synth.FFT_CONFIGS:
        run_fftdf(args, dev)
        return
    wl = synth.BN33 if args.config == "bn33" else synth.CONFIGS[args.config]
    imp_idx, val_idx = synth.bn33_impurity() if args.config == "bn33" else (None, None)
    print(f"[bench] generating {wl.name} inputs", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    lat = synth.make_lattice(wl)
    lm = synth.three_index(wl)
    t_gen = time.perf_counter() - t0
    print(f"[bench] inputs generated in {t_gen:.1f} s; copying {lm.nbytes / 1e9:.1f} GB to HBM",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    lm_d = torch.from_numpy(lm).to(dev)
    torch.cuda.synchronize()
    t_h2d = time.perf_counter() - t0
    dm_d = torch.from_numpy(lat.dm_k).to(dev)
    h_d = torch.from_numpy(lat.h_k).to(dev)

    # bath + one-body (not in the timed region); the second, warm pass is the one timed
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for _ in range(2):
        ev[0].record()
        ck, sv, neo = dmet.dmet_build_bath(wl.kmesh, wl.nao, dm_d, imp_idx=imp_idx, val_idx=val_idx)
        ev[1].record()
        h_eo, _ = dmet.dmet_transform_1e(wl.kmesh, wl.nao, ck, h_d)
        g_eo, _ = dmet.dmet_transform_1e(wl.kmesh, wl.nao, ck, dm_d)
        e1 = dmet.dmet_energy_1e(h_eo, g_eo)
        ev[2].record()
        torch.cuda.synchronize()
    t_bath = ev[0].elapsed_time(ev[1])
    t_1e = ev[1].elapsed_time(ev[2])
    print(f"[bench] bath {t_bath:.2f} ms, one-body {t_1e:.2f} ms, E1 = {float(e1.cpu()):.10f}",
          file=sys.stderr, flush=True)

    def full_step(prec, ws, out):
        # one pass of the whole path: bath and C^k, one-body h and gamma, E1, ERIs
        ck_s, _, _ = dmet.dmet_build_bath(wl.kmesh, wl.nao, dm_d, imp_idx=imp_idx, val_idx=val_idx)
        h_s, _ = dmet.dmet_transform_1e(wl.kmesh, wl.nao, ck_s, h_d)
        g_s, _ = dmet.dmet_transform_1e(wl.kmesh, wl.nao, ck_s, dm_d)
        dmet.dmet_energy_1e(h_s, g_s)
        mid = torch.cuda.Event(enable_timing=True)
        mid.record(torch.cuda.current_stream())
        return mid, dmet.dmet_transform_eri(wl.kmesh, wl.nao, wl.naux, lm_d, ck_s, prec, workspace=ws, out=out)

    def run_form(prec, steps, warmup, keep=False):
        ws = torch.empty(dmet.dmet_transform_eri_workspace(wl.kmesh, wl.nao, wl.naux, wl.nspin, wl.neo, prec,
                                                           lm_d.dtype), dtype=torch.uint8, device=dev)
        out = None
        for _ in range(warmup):
            _, out = full_step(prec, ws, out)
        torch.cuda.synchronize()
        dmet.dmet_profile_reset()
        dmet.dmet_profile_enable(True)
        st = torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        mids = []
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        ev[0].record(st)
        for n in range(steps):
            mid, out = full_step(prec, ws, out)
            mids.append(mid)
            ev[n + 1].record(st)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        dmet.dmet_profile_enable(False)
        prof = dmet.dmet_profile_report()
        ms = ev[0].elapsed_time(ev[steps]) / steps
        eri_ms = sum(mids[n].elapsed_time(ev[n + 1]) for n in range(steps)) / steps
        del ws
        if not keep:
            out = None
        return ms, wall, prof, out, eri_ms

    forms = [args.precision] + [p for p in args.compare.split(",") if p and p != args.precision]
    # FP64 first (when compared), so that each other form is checked against it
    # as soon as it has run and only the FP64 output is kept
    order = (["fp64"] if "fp64" in forms else []) + [p for p in forms if p != "fp64"]
    results, checks = {}, {}
    for prec in order:
        print(f"[bench] timing {prec}: warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
        ms, wall, prof, out, eri_ms = run_form(prec, args.steps, args.warmup, keep=len(forms) > 1)
        if out is not None:
            chk = {"E": coulomb_exchange_energies(out, g_eo)}
            if prec != "fp64" and "fp64" in results:
                ref = results["fp64"][3]
                chk["max_abs_err_vs_fp64"] = {k: float((out[k] - ref[k]).abs().max()) for k in out}
            checks[prec] = chk
            if prec != "fp64":
                out = None
                torch.cuda.empty_cache()
        results[prec] = (ms, wall, prof, out, eri_ms)
        print(f"[bench] {prec}: {ms:.2f} ms/step ({eri_ms:.2f} ms ERI build); kernels {prof}; "
              f"{checks.get(prec, {})}", file=sys.stderr, flush=True)

    # next rows: density-fitting output (contraction skipped) and the
    # double-counting-corrected Fock matrix from it, timed once each
    f_d = torch.from_numpy(lat.f_k).to(dev)
    f_eo, _ = dmet.dmet_transform_1e(wl.kmesh, wl.nao, ck, f_d)
    ws_df = torch.empty(dmet.dmet_transform_eri_workspace(wl.kmesh, wl.nao, wl.naux, wl.nspin, wl.neo,
                                                          args.precision, lm_d.dtype), dtype=torch.uint8, device=dev)
    z = dmet.dmet_transform_eri_df(wl.kmesh, wl.nao, wl.naux, lm_d, ck, args.precision, workspace=ws_df)
    dmet.dmet_fock_dc(z, f_eo, g_eo)
    torch.cuda.synchronize()
    ev2 = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev2[0].record()
    z = dmet.dmet_transform_eri_df(wl.kmesh, wl.nao, wl.naux, lm_d, ck, args.precision, workspace=ws_df)
    ev2[1].record()
    ft = dmet.dmet_fock_dc(z, f_eo, g_eo)
    e_mf = dmet.dmet_energy_mf(ft, f_eo, g_eo)
    ev2[2].record()
    torch.cuda.synchronize()
    t_df, t_dc = ev2[0].elapsed_time(ev2[1]), ev2[1].elapsed_time(ev2[2])
    print(f"[bench] DF output {t_df:.2f} ms, double-counting Fock and mean-field energy {t_dc:.2f} ms "
          f"(E_mf = {float(e_mf.cpu()):.10f})", file=sys.stderr, flush=True)
    del z, ws_df, ft
    hbm_tbs = hbm_copy_rate(dev)

    wt, wc = work_counts(wl)
    ms, wall, prof, _, eri_ms = results[args.precision]
    # The paper quotes ~200 s for this shape's embedding ERIs on 28 Xeon cores
    # (Sec. 2.1, after Alg. 1); only that workload has a paper number.
    paper_s = 200.0 if args.config == "bn33" else None
    value = (wt + wc) / (ms * 1e-3) / 1e12
    # dominant kernel: largest total time in the timed region
    dom = max(prof.items(), key=lambda kv: kv[1][1])
    dname, (dn, dms) = dom
    avg_ms = dms / dn
    kf = kernel_flops(wl, dname)
    achieved = kf / (avg_ms * 1e-3) / 1e12
    line = {
        "metric": METRIC, "value": round(value, 4), "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None if paper_s is None else round(paper_s / (ms * 1e-3), 1),
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: k-mesh {'x'.join(map(str, wl.kmesh))}, nao {wl.nao}, naux {wl.naux}, "
                               f"neo {wl.neo}, nspin {wl.nspin}, 3-index {'complex128' if lm.dtype == np.complex128 else 'complex64'}",
                   "precision": args.precision, "W_flop": wt + wc, "W_T": wt, "W_C": wc},
        "roofline": {"bound": "mfma", "kernel": dname, "achieved": round(achieved, 3),
                     "peak": kernel_peak(args.precision, dname),
                     "unit": "TFLOP/s", "frac": round(achieved / kernel_peak(args.precision, dname), 4),
                     "traffic": traffic_bytes(dname, wl.name),
                     "mfma_util": round(achieved * MFMA_PRODUCTS[args.precision] / kernel_peak(args.precision, dname),
                                        4),
                     "launch_ms": round(avg_ms, 4), "flop_per_launch": kf},
        "eri_build_ms": round(eri_ms, 3),
        "kernels_ms_per_step": {k: round(v[1] / args.steps, 3) for k, v in prof.items()},
        # every ERI kernel with an algorithmic flop count, on the same convention as `roofline`
        "rooflines": {k: {"launches_per_step": round(n / args.steps, 2), "launch_ms": round(t / n, 4),
                          "achieved": round(kernel_flops(wl, k) / (t / n * 1e-3) / 1e12, 3),
                          "peak": kernel_peak(args.precision, k),
                          "frac": round(kernel_flops(wl, k) / (t / n * 1e-3) / 1e12 / kernel_peak(args.precision, k), 4),
                          "traffic": traffic_bytes(k, wl.name)}
                      for k, (n, t) in prof.items() if kernel_flops(wl, k) is not None and n > 0},
        "bath_ms": round(t_bath, 3), "onebody_ms": round(t_1e, 3),
        "df_output_ms": round(t_df, 3), "fock_dc_ms": round(t_dc, 3),
        "h2d_s": round(t_h2d, 2), "h2d_GBps": round(lm.nbytes / 1e9 / t_h2d, 2),
        "hbm_copy_TBs_measured": hbm_tbs,
    }
    if len(forms) > 1:
        cmp = {}
        e64 = checks.get("fp64", {}).get("E")
        for prec in forms:
            msp = results[prec][0]
            entry = {"ms_per_step": round(msp, 3), "eri_build_ms": round(results[prec][4], 3),
                     "TFLOP/s": round((wt + wc) / (msp * 1e-3) / 1e12, 3)}
            chk = checks.get(prec, {})
            if "E" in chk:
                entry["E_J_E_K"] = chk["E"]
                if e64 is not None and prec != "fp64":
                    entry["E_err_vs_fp64"] = {k: {n: abs(v - e64[k][n]) for n, v in d.items()}
                                              for k, d in chk["E"].items()}
            if "max_abs_err_vs_fp64" in chk:
                entry["max_abs_err_vs_fp64"] = chk["max_abs_err_vs_fp64"]
                entry["speedup_vs_fp64"] = round(results["fp64"][0] / msp, 3)
            cmp[prec] = entry
        line["forms"] = cmp
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        n_l = args.cpu_sample_l or max(1, wl.naux // 2)
        line["cpu_baseline"] = cpu_baseline(wl, lat, lm, min(n_l, wl.naux),
                                            min(args.cpu_sample_rows, wl.neo * wl.neo), imp_idx, val_idx,
                                            w_flop=wt + wc, one_thread=wl.name in ("tiny", "hbn"))
        model, mem = host_info()
        line["cpu_baseline"]["host"] = {"model": model, "os_cpu_count": os.cpu_count(), "ram_gb": mem}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
