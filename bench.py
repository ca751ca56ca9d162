#!/usr/bin/env python3
"""Benchmark of the (ab|cd) hot path on one MI355X.

A step is one eri4_batch call over the whole batch: Boys function, Hermite
integrals, both Hermite-to-Cartesian MFMA transforms and the output write, for
512 (ii|ii) quartets (l = 6, Cartesian, 784 x 784 integrals each) with inputs
already resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload iiii_k1|iiii_k5|gggg_k1]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6  # MI355X published dense FP64 (vector and matrix)
METRIC = "(ii|ii) integrals/s + % FP64 peak; mixed-prec vs FP64 speedup at ≤1e-10 err"
KERNEL = "eri4_fused_kernel"
# the files that define eri4_fused_kernel (its traffic counters hold while they are unchanged)
SOURCES = ["paper_2307_03452_amd/csrc/" + f for f in
           ("eri4_device.h", "eri4_internal.h", "eri4_launch.h", "eri4_fused.hip")]

WORKLOADS = {
    "iiii_k1": dict(ls=(6, 6, 6, 6), K=1, nq=512, seed=1002, exps=(0.05, 200.0),
                    desc="(ii|ii) l=6 Cartesian, K=1 per shell, 512 quartets, exponents log-uniform [0.05,200], "
                         "centres uniform in an 8-Bohr cube, unit-normalised shells, FP64 out [512][28][28][28][28]"),
    "iiii_k5": dict(ls=(6, 6, 6, 6), K=5, nq=512, seed=1003, exps=(0.05, 200.0),
                    desc="(ii|ii) l=6 Cartesian, K=5 per shell (K_bra=K_ket=25), coefficients U[0.1,1], 512 quartets, "
                         "exponents log-uniform [0.05,200], 8-Bohr cube, FP64 out"),
    "gggg_k1": dict(ls=(4, 4, 4, 4), K=1, nq=64, seed=1001, exps=(0.05, 50.0),
                    desc="(gg|gg) l=4 Cartesian, K=1, 64 quartets, exponents log-uniform [0.05,50], 8-Bohr cube"),
}


def source_hash() -> str:
    h = hashlib.sha256()
    for s in SOURCES:
        with open(os.path.join(ROOT, s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload: str):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{KERNEL}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_sha256") != source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def make_batch(wl):
    from paper_2307_03452_amd import inputs
    return inputs.class_batch(wl["ls"], wl["nq"], wl["K"], seed=wl["seed"], exp_range=wl["exps"])


def time_gpu(wl, b, steps, warmup):
    import torch
    from paper_2307_03452_amd import eri4, metrics
    d = lambda a: torch.from_numpy(a).cuda()
    C, E, Co, N = d(b.centers), d(b.exps), d(b.coefs), d(b.nprim)
    ls = wl["ls"]
    out = torch.empty((b.nq,) + tuple(metrics.ncart(l) for l in ls), dtype=torch.float64, device="cuda")
    eri4.init()
    for _ in range(warmup):
        eri4.batch(ls, C, E, Co, N, out=out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(stream)
        eri4.batch(ls, C, E, Co, N, out=out, stream=stream)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = [a.elapsed_time(z) for a, z in ev]
    return out, wall, launch_ms


def md4_flops_batch(lq, nprim):
    from paper_2307_03452_amd import metrics
    tot = 0
    for (la, lb, lc, ld), k in zip(lq.tolist(), nprim.tolist()):
        tot += metrics.md4_flops(la, lb, lc, ld, k[0] * k[1], k[2] * k[3])
    return tot


TUNE_FILE = os.path.join(ROOT, "paper_2307_03452_amd", "tune_gfx950.txt")


def tuned_tiles():
    """The autotuner's tile table (paper_2307_03452_amd/autotune.py) as tile
    choices, for the pair-list plans; quartet plans read the file through the
    library (tune_file)."""
    if not os.path.exists(TUNE_FILE):
        return None
    from paper_2307_03452_amd import eri4
    return eri4.read_tile_table(TUNE_FILE)


def time_plan(b, precision, steps, warmup, tiles=None, tune_file=None):
    """One plan over batch b (inputs resident in HBM): wall seconds per execute."""
    import torch
    from paper_2307_03452_amd import eri4
    plan = eri4.Plan(b.lq, b.nprim, b.kmax, precision=precision, tiles=tiles, tune_file=tune_file)
    d = lambda a: torch.from_numpy(a).cuda()
    C, E, Co = d(b.centers), d(b.exps), d(b.coefs)
    out = torch.empty(plan.output_size, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        plan.execute(C, E, Co, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.execute(C, E, Co, out=out)
    torch.cuda.synchronize()
    return plan, out, (time.perf_counter() - t0) / steps


def sampled_oracle_err(b, plan, out, absolute=False, smallest=False):
    """Largest error against the oracle over a few quartets of batch b,
    relative to each quartet's largest integral, or absolute.  The sample: the
    quartet with the largest total l and three random ones among quartets whose
    four contraction lengths multiply to at most 16 (which the oracle does
    quickly); with smallest=True, the two with the smallest total l and one
    random one among those with total l <= 17."""
    import oracle
    from paper_2307_03452_amd import inputs
    off = plan.offsets()
    rng = np.random.default_rng(7)
    if smallest:
        tot = b.lq.sum(axis=1)
        small = np.flatnonzero(tot <= 17)
        idx = sorted({*np.argsort(tot, kind="stable")[:2].tolist(), int(rng.choice(small))})
    else:
        cheap = np.flatnonzero(np.prod(b.nprim, axis=1) <= 16)
        big = cheap[np.argmax(b.lq[cheap].sum(axis=1))]
        idx = sorted({int(big), *rng.choice(cheap, 3, replace=False).tolist()})
    err = 0.0
    for q in idx:
        s_ = inputs.subset(b, [q])
        o = oracle.eri_md4(tuple(int(x) for x in b.lq[q]), s_.centers, s_.exps, s_.coefs, s_.nprim)[0]
        g = out[off[q]:off[q] + o.size].cpu().numpy().reshape(o.shape)
        e = float(np.abs(g - o).max())
        err = max(err, e if absolute else e / max(np.abs(o).max(), 1e-250))
    return err


UNEVEN_DESC = ("uneven batch: {nq} quartets, 81 classes (la lb|lc ld) in {{4,5,6}}^4 with Zipf(1.2) counts, "
               "K per shell uniform in 1..8, exponents [0.05,200], one persistent launch")


def time_uneven(steps, warmup, nq=20000, seed=1004, mixed_steps=0):
    """Uneven batch in one persistent launch: all ordered classes in {4,5,6}^4,
    Zipf(1.2) class counts, contraction length 1..8 per shell.  With
    mixed_steps > 0 the same batch also runs with FP32 transforms."""
    from paper_2307_03452_amd import inputs
    b = inputs.uneven_batch(nq=nq, seed=seed)
    tf = TUNE_FILE if os.path.exists(TUNE_FILE) else None
    plan, out, wall = time_plan(b, "fp64", steps, warmup, tune_file=tf)
    flops = md4_flops_batch(b.lq, b.nprim)
    rec = {"workload": UNEVEN_DESC.format(nq=nq),
           "value": plan.output_size / wall, "unit": "integrals/s", "ms_per_step": wall * 1e3,
           "md4_tflops": flops / wall / 1e12, "pct_fp64_peak": 100 * flops / wall / 1e12 / FP64_PEAK_TFLOPS,
           "parity_max_rel_err_sampled": sampled_oracle_err(b, plan, out), "quartets": nq,
           "tiles": "autotuned table (tune_gfx950.txt, read by eri4_plan_create_tunefile)" if tf else "library default"}
    mixed = None
    if mixed_steps > 0:
        plan32, out32, wall32 = time_plan(b, "fp32", mixed_steps, 1, tune_file=tf)
        mixed = {"workload": UNEVEN_DESC.format(nq=nq), "precision": "fp32",
                 "transforms": "operands rounded to FP32, FP32 matrix cores, FP32 accumulation; "
                               "Boys, R and E in FP64",
                 "value": plan32.output_size / wall32, "unit": "integrals/s", "ms_per_step": wall32 * 1e3,
                 "fp64_ms_per_step": wall * 1e3, "speedup_vs_fp64": wall / wall32,
                 "oracle_max_abs_err_sampled": sampled_oracle_err(b, plan32, out32, absolute=True)}
        mixed.update(class_errors(b, plan, out, out32))
        del out32
    return rec, mixed


def time_classes_l7(reps=1):
    """(kk|kk) and (ik|ik), K=3 per shell, 256 quartets each: eri4_batch (FP64)
    and a one-class plan with FP32 transforms."""
    import torch
    from paper_2307_03452_amd import eri4, inputs, metrics
    d = lambda a: torch.from_numpy(a).cuda()
    out = []
    for ls, seed in (((7, 7, 7, 7), 1005), ((6, 7, 6, 7), 1007)):
        b = inputs.class_batch(ls, 256, 3, seed=seed, exp_range=(0.05, 200.0))
        C, E, Co, N = d(b.centers), d(b.exps), d(b.coefs), d(b.nprim)
        o = eri4.batch(ls, C, E, Co, N)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            eri4.batch(ls, C, E, Co, N, out=o)
        torch.cuda.synchronize()
        t64 = (time.perf_counter() - t0) / reps
        b.lq = np.tile(np.array(ls, np.int32), (b.nq, 1))
        _, o32, t32 = time_plan(b, "fp32", reps, 1, tune_file=TUNE_FILE if os.path.exists(TUNE_FILE) else None)
        err = float((o32 - o.reshape(-1)).abs().max())
        flops = b.nq * metrics.md4_flops(*ls, 9, 9)
        ints = b.nq * metrics.integrals_per_quartet(*ls)
        out.append({"class": "(%d%d|%d%d)" % ls, "quartets": b.nq, "K_per_shell": 3,
                    "value": ints / t64, "unit": "integrals/s", "ms_per_step": t64 * 1e3,
                    "pct_fp64_peak": 100 * flops / t64 / 1e12 / FP64_PEAK_TFLOPS,
                    "fp32_speedup_vs_fp64": t64 / t32, "fp32_max_abs_err_vs_fp64": err})
        del o, o32
    return out


def time_low_l(nq=4096, reps=3):
    """(dd|dd) and (ff|ff) at the paper's K = K_bra K_ket in {1, 5, 25}: one
    eri4_batch call per case, inputs resident, 4096 quartets each."""
    import torch
    from paper_2307_03452_amd import eri4, inputs, metrics
    d = lambda a: torch.from_numpy(a).cuda()
    out = []
    for l in (2, 3):
        for K in (1, 5, 25):
            b = inputs.low_l_batch(l, K, nq, seed=1100 + 10 * l + K)
            C, E, Co, N = d(b.centers), d(b.exps), d(b.coefs), d(b.nprim)
            o = eri4.batch(b.ls, C, E, Co, N)
            torch.cuda.synchronize()
            # more back-to-back calls for the short cases (60 at K = 1), so
            # that one call's launch latency does not weigh on a 0.07 ms kernel
            n = max(reps, 60 // K)
            t0 = time.perf_counter()
            for _ in range(n):
                eri4.batch(b.ls, C, E, Co, N, out=o)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / n
            ks = inputs.PAPER_K_SHELLS[K]
            flops = nq * metrics.md4_flops(l, l, l, l, ks[0] * ks[1], ks[2] * ks[3])
            ints = nq * metrics.integrals_per_quartet(l, l, l, l)
            out.append({"class": "(%s%s|%s%s)" % ((("d", "f")[l - 2],) * 4), "K_bra_K_ket": K,
                        "contraction_lengths": list(ks), "quartets": nq, "calls_timed": n, "value": ints / t,
                        "unit": "integrals/s", "ms_per_step": t * 1e3,
                        "pct_fp64_peak": 100 * flops / t / 1e12 / FP64_PEAK_TFLOPS,
                        "hbm_gb_per_s_output": nq * metrics.output_bytes(l, l, l, l) / t / 1e9})
            del o
    return out


def time_pairs(nbra=128, nket=128, kmax=3, reps=3):
    """Bra list x ket list (eri4_plan_*_pairs): 128 x 128 shell pairs with l in
    {4,5,6} per shell and contraction lengths 1..3, against the quartet plan
    over the expanded batch (same quartets, per-quartet shell arrays)."""
    import torch
    from paper_2307_03452_amd import eri4, inputs, metrics
    bra, ket = inputs.pair_list(nbra, 1201, kmax=kmax), inputs.pair_list(nket, 1202, kmax=kmax)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    tiles = tuned_tiles()
    pp = eri4.PairPlan(bra.l, bra.nprim, ket.l, ket.nprim, kmax, tiles=tiles)
    args = (d(bra.centers), d(bra.exps), d(bra.coefs), d(ket.centers), d(ket.exps), d(ket.coefs))
    out = pp.execute(*args)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        pp.execute(*args, out=out)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    # the same lists over real solid harmonics: H once per list entry
    ps = eri4.PairPlan(bra.l, bra.nprim, ket.l, ket.nprim, kmax, tiles=tiles, functions="solid")
    work = torch.empty(max(1, ps.work_size), dtype=torch.float64, device="cuda")
    sout = ps.execute(*args, work=work)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ps.execute(*args, out=sout, work=work)
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / reps
    b = inputs.expand_pairs(bra, ket)
    sflops = sum(metrics.md4_flops(*(int(x) for x in b.lq[q]), int(b.nprim[q, 0] * b.nprim[q, 1]),
                                   int(b.nprim[q, 2] * b.nprim[q, 3]), solid=True) for q in range(b.nq))
    solid_rec = {"value": ps.output_size / ts, "unit": "integrals/s", "ms_per_step": ts * 1e3,
                 "pct_fp64_peak": 100 * sflops / ts / 1e12 / FP64_PEAK_TFLOPS, "workspace_bytes": ps.work_size * 8}
    del work, sout
    # Coulomb contraction over the same lists: J of every bra entry
    rng = np.random.default_rng(1203)
    kd = d(np.concatenate([rng.uniform(-1.0, 1.0, size=metrics.ncart(int(ket.l[j, 0])) * metrics.ncart(int(ket.l[j, 1])))
                           for j in range(nket)]))
    pc = eri4.CoulombPlan(bra.l, bra.nprim, ket.l, ket.nprim, kmax)
    cwork = torch.empty(max(1, pc.work_size), dtype=torch.float64, device="cuda")
    cout = pc.execute(*args, kd, work=cwork)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        pc.execute(*args, kd, out=cout, work=cwork)
    torch.cuda.synchronize()
    tc = (time.perf_counter() - t0) / reps
    coul_rec = {"ms_per_step": tc * 1e3, "integrals_contracted_per_s": pp.output_size / tc,
                "output_bytes": pc.output_size * 8, "workspace_bytes": pc.work_size * 8}
    del cwork, cout
    _, qout, tq = time_plan(b, "fp64", reps, 1, tiles)
    flops = md4_flops_batch(b.lq, b.nprim)
    return {"workload": "bra list x ket list: %d x %d shell pairs, l in {4,5,6} per shell, K per shell 1..%d"
                        % (nbra, nket, kmax),
            "quartets": b.nq, "value": pp.output_size / t, "unit": "integrals/s", "ms_per_step": t * 1e3,
            "pct_fp64_peak": 100 * flops / t / 1e12 / FP64_PEAK_TFLOPS,
            "quartet_plan_ms_per_step": tq * 1e3, "bitwise_equal_to_quartet_plan": bool(torch.equal(out, qout)),
            "input_bytes": int(sum(a.numel() * 8 for a in args)),
            "quartet_plan_input_bytes": int((b.centers.size + b.exps.size + b.coefs.size) * 8),
            "solid": solid_rec, "coulomb": coul_rec}


def time_solid(reps=3):
    """Solid-harmonic output (eri4_batch_solid, FP64): (ii|ii) K=1 on the
    512-quartet batch and K=5 per shell on its first 128 quartets.  FLOPs are
    the two transforms over solid functions, 2 Sab (Kb Np)(Kk Nq) + 2 Sab (Kk Nq) Scd
    per quartet; the time includes building the H matrices."""
    import torch
    from paper_2307_03452_amd import eri4, inputs, metrics
    from oracle import solid
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    out = []
    for K, nq in ((1, 512), (5, 128)):
        b = inputs.subset(inputs.iiii(K=K), range(nq))
        C, E, Co, N = d(b.centers), d(b.exps), d(b.coefs), d(b.nprim)
        work = torch.empty(eri4.solid_work_size(b.ls, b.kmax, nq), dtype=torch.float64, device="cuda")
        o = eri4.batch_solid(b.ls, C, E, Co, N, work=work)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            eri4.batch_solid(b.ls, C, E, Co, N, work=work, out=o)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        flops = nq * metrics.md4_flops(6, 6, 6, 6, K * K, K * K, solid=True)
        # parity: two quartets against the oracle, relative to the scale the
        # transform rounds at, max sum_k |C x C x C x C|[m, k] |cart[k]|
        import oracle
        cart = oracle.eri_md4(b.ls, b.centers[:2], b.exps[:2], b.coefs[:2], b.nprim[:2])
        ref = solid.cart_to_solid(cart, b.ls)
        bound = solid.cart_to_solid(np.abs(cart), b.ls, absolute=True)
        g = o[:2].cpu().numpy()
        err = max(float(np.abs(g[i] - ref[i]).max() / bound[i].max()) for i in range(2))
        out.append({"workload": "(ii|ii) solid harmonics, K=%d per shell, %d quartets" % (K, nq),
                    "value": nq * 13 ** 4 / t, "unit": "integrals/s", "ms_per_step": t * 1e3,
                    "pct_fp64_peak": 100 * flops / t / 1e12 / FP64_PEAK_TFLOPS,
                    "workspace_bytes": work.numel() * 8, "parity_max_err_2q_rel_transform_bound": err})
        del work, o
    # a quartet plan over solid harmonics (mixed classes, one persistent
    # launch after the H build) beside the Cartesian plan on the same quartets
    nq = 1024
    b = inputs.stream_batch(nq, 1006)
    C, E, Co = d(b.centers), d(b.exps), d(b.coefs)
    tf = TUNE_FILE if os.path.exists(TUNE_FILE) else None
    times = {}
    for kind in ("solid", "cartesian"):
        p = (eri4.SolidPlan(b.lq, b.nprim, b.kmax, tune_file=tf) if kind == "solid"
             else eri4.Plan(b.lq, b.nprim, b.kmax, tune_file=tf))
        work = (torch.empty(max(1, p.work_size), dtype=torch.float64, device="cuda") if kind == "solid" else None)
        o = p.execute(C, E, Co, work=work) if work is not None else p.execute(C, E, Co)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            if work is not None:
                p.execute(C, E, Co, out=o, work=work)
            else:
                p.execute(C, E, Co, out=o)
        torch.cuda.synchronize()
        times[kind] = (time.perf_counter() - t0) / reps
        if work is not None:
            wbytes = work.numel() * 8
        del o, work, p
    flops = sum(metrics.md4_flops(*(int(x) for x in b.lq[q]), int(b.nprim[q, 0] * b.nprim[q, 1]),
                                  int(b.nprim[q, 2] * b.nprim[q, 3]), solid=True) for q in range(nq))
    ints = sum(int(np.prod([2 * int(x) + 1 for x in b.lq[q]])) for q in range(nq))
    out.append({"workload": f"solid quartet plan: {nq} quartets, classes in {{4,5,6,7}}^4 (Zipf(1.2) counts), "
                            "K=3 per shell, one persistent launch after the H build",
                "value": ints / times["solid"], "unit": "integrals/s", "ms_per_step": times["solid"] * 1e3,
                "pct_fp64_peak": 100 * flops / times["solid"] / 1e12 / FP64_PEAK_TFLOPS,
                "cartesian_plan_ms_per_step": times["cartesian"] * 1e3, "workspace_bytes": wbytes})
    return out


def time_gggg(graph_calls=100, reps=5):
    """(gg|gg) K=1, 64 quartets (2.9e7 MD4 FLOPs each; 24 us at FP64 peak, so
    launch overhead matters): one eri4_batch call timed with HIP events on its
    stream, and a HIP graph of 100 calls replayed (time per call)."""
    import torch
    from paper_2307_03452_amd import eri4, inputs, metrics
    wl = WORKLOADS["gggg_k1"]
    b = make_batch(wl)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    C, E, Co, N = d(b.centers), d(b.exps), d(b.coefs), d(b.nprim)
    out = eri4.batch(b.ls, C, E, Co, N)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    single = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        eri4.batch(b.ls, C, E, Co, N, out=out, stream=s)
        e1.record(s)
        torch.cuda.synchronize()
        single.append(e0.elapsed_time(e1))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for _ in range(graph_calls):
            eri4.batch(b.ls, C, E, Co, N, out=out, stream=s)
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        with torch.cuda.stream(s):
            g.replay()
    e1.record(s)
    torch.cuda.synchronize()
    per_call = e0.elapsed_time(e1) / (reps * graph_calls)
    flops = b.nq * metrics.md4_flops(4, 4, 4, 4, 1, 1)
    ints = b.nq * metrics.integrals_per_quartet(4, 4, 4, 4)
    t1 = sorted(single)[len(single) // 2]
    return {"workload": wl["desc"], "single_launch_ms": t1, "single_pct_fp64_peak": 100 * flops / t1 / 1e9 / FP64_PEAK_TFLOPS,
            "graph_calls": graph_calls, "graph_ms_per_call": per_call,
            "graph_pct_fp64_peak": 100 * flops / per_call / 1e9 / FP64_PEAK_TFLOPS,
            "value": ints / (per_call / 1e3), "unit": "integrals/s"}


def time_coulomb(reps=3):
    """Coulomb contraction without forming (ab|cd) (eri4_batch_coulomb): (ii|ii)
    K=1 on the 512-quartet batch and K=5 per shell on its first 128 quartets,
    next to forming the same integrals.  FLOPs performed (J-engine order):
    the density to Hermite space 2 Kk Nq Ncd, the matrix-vector products with
    [p+q] 2 Kb Kk Np Nq, and the bra transform 2 Kb Nab Np, all on the vector
    units; the rate is quoted against the FP64 peak (78.6 TFLOP/s, which the
    vector units share with the matrix cores on this part)."""
    import torch
    from paper_2307_03452_amd import eri4, inputs, metrics
    import oracle
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    out = []
    for K, nq in ((1, 512), (5, 128)):
        b = inputs.subset(inputs.iiii(K=K), range(nq))
        D = inputs.ket_densities(b, seed=1300 + K)
        C, E, Co, N, Dd = d(b.centers), d(b.exps), d(b.coefs), d(b.nprim), d(D)
        work = torch.empty(eri4.coulomb_work_size(b.ls, b.kmax, nq), dtype=torch.float64, device="cuda")
        o = eri4.batch_coulomb(b.ls, C, E, Co, N, Dd, work=work)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            eri4.batch_coulomb(b.ls, C, E, Co, N, Dd, work=work, out=o)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        # the integrals themselves on the same batch, for comparison
        ints = eri4.batch(b.ls, C, E, Co, N)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            eri4.batch(b.ls, C, E, Co, N, out=ints)
        torch.cuda.synchronize()
        t_ints = (time.perf_counter() - t0) / reps
        del ints
        kb = K * K
        npp = metrics.nherm(12)
        flops = nq * (2 * kb * npp * 784 + 2 * kb * kb * npp * npp + 2 * kb * 784 * npp)
        I = oracle.eri_md4(b.ls, b.centers[:2], b.exps[:2], b.coefs[:2], b.nprim[:2])
        ref = np.einsum("qabcd,qcd->qab", I, D[:2])
        bound = np.einsum("qabcd,qcd->qab", np.abs(I), np.abs(D[:2]))
        g = o[:2].cpu().numpy()
        err = max(float(np.abs(g[i] - ref[i]).max() / bound[i].max()) for i in range(2))
        out.append({"workload": "(ii|ii) Coulomb contraction J_ab = sum_cd (ab|cd) D_cd, K=%d per shell, %d quartets"
                                % (K, nq), "ms_per_step": t * 1e3, "integrals_ms_per_step_same_batch": t_ints * 1e3,
                    "speedup_vs_forming_integrals": t_ints / t,
                    "flops_performed": flops, "pct_fp64_peak": 100 * flops / t / 1e12 / FP64_PEAK_TFLOPS,
                    "output_bytes": nq * 784 * 8, "integrals_contracted_per_s": nq * 784 * 784 / t,
                    "parity_max_err_2q_rel_contraction_bound": err})
        del work, o
    return out


def time_exchange(reps=3):
    """Exchange contraction without forming (ab|cd) (eri4_batch_exchange):
    (ii|ii) K=1 on the 512-quartet batch and K=5 per shell on its first 128
    quartets, next to forming the same integrals.  FLOPs: the first transform
    2 Nab' (Kb Np)(Kk Nq) over the padded bra rows Nab' = Nb 16 ceil(Na/16), and
    the contraction with F^b 2 Nab' Kk Nq Nc; F^b itself costs
    2 Kk Nb Nq Nc Nd on the vector units."""
    import torch
    from paper_2307_03452_amd import eri4, inputs, metrics
    import oracle
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    out = []
    for K, nq in ((1, 512), (5, 128)):
        b = inputs.subset(inputs.iiii(K=K), range(nq))
        D = inputs.exchange_densities(b, seed=1500 + K)
        C, E, Co, N, Dd = d(b.centers), d(b.exps), d(b.coefs), d(b.nprim), d(D)
        work = torch.empty(eri4.exchange_work_size(b.ls, b.kmax, nq), dtype=torch.float64, device="cuda")
        o = eri4.batch_exchange(b.ls, C, E, Co, N, Dd, work=work)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            eri4.batch_exchange(b.ls, C, E, Co, N, Dd, work=work, out=o)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        ints = eri4.batch(b.ls, C, E, Co, N)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            eri4.batch(b.ls, C, E, Co, N, out=ints)
        torch.cuda.synchronize()
        t_ints = (time.perf_counter() - t0) / reps
        del ints
        kb = K * K
        npp = metrics.nherm(12)
        rows = 28 * 32
        flops = nq * (2 * rows * (kb * npp) * (kb * npp) + 2 * rows * kb * npp * 28)
        I = oracle.eri_md4(b.ls, b.centers[:2], b.exps[:2], b.coefs[:2], b.nprim[:2])
        ref = np.einsum("qabcd,qbd->qac", I, D[:2])
        bound = np.einsum("qabcd,qbd->qac", np.abs(I), np.abs(D[:2]))
        g = o[:2].cpu().numpy()
        err = max(float(np.abs(g[i] - ref[i]).max() / bound[i].max()) for i in range(2))
        out.append({"workload": "(ii|ii) exchange contraction K_ac = sum_bd (ab|cd) D_bd, K=%d per shell, %d quartets"
                                % (K, nq), "ms_per_step": t * 1e3, "integrals_ms_per_step_same_batch": t_ints * 1e3,
                    "speedup_vs_forming_integrals": t_ints / t,
                    "pct_fp64_peak": 100 * flops / t / 1e12 / FP64_PEAK_TFLOPS,
                    "output_bytes": nq * 28 * 28 * 8, "integral_bytes_not_written": nq * 784 * 784 * 8,
                    "workspace_bytes": work.numel() * 8,
                    "integrals_contracted_per_s": nq * 784 * 784 / t,
                    "parity_max_err_2q_rel_contraction_bound": err})
        del work, o
    return out


def time_stream(nq=50000, seed=1006, chunk=1024, ring=4):
    """Serving-style stream: 50 000 quartets over the 256 classes in {4..7}^4
    (Zipf counts, K=3 per shell) in chunks of 1024, each chunk a HIP graph
    (the plan's counter reset and persistent kernel) replayed into a ring of
    output buffers; FP64 and FP32 transforms."""
    import torch
    from paper_2307_03452_amd import eri4, inputs
    b = inputs.stream_batch(nq, seed)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    C, E, Co = d(b.centers), d(b.exps), d(b.coefs)
    starts = list(range(0, nq, chunk))
    views = [(C[s0:s0 + chunk], E[s0:s0 + chunk], Co[s0:s0 + chunk]) for s0 in starts]
    flops = md4_flops_batch(b.lq, b.nprim)
    rec = {"workload": f"stream of {nq} quartets, 256 classes (la lb|lc ld) in {{4,5,6,7}}^4 with Zipf(1.2) counts, "
                       f"K=3 per shell, exponents [0.05,200]; chunks of {chunk} quartets, each a HIP graph replayed "
                       f"into a ring of {ring} output buffers", "chunks": len(starts)}
    check = {}
    for prec in ("fp64", "fp32"):
        tf = TUNE_FILE if os.path.exists(TUNE_FILE) else None
        plans = [eri4.Plan(b.lq[s0:s0 + chunk], b.nprim[s0:s0 + chunk], b.kmax, precision=prec, tune_file=tf)
                 for s0 in starts]
        size = max(p.output_size for p in plans)
        outs = [torch.empty(size, dtype=torch.float64, device="cuda") for _ in range(ring)]
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        plans[0].execute(*views[0], out=outs[0], stream=side)  # first use of the device outside capture
        torch.cuda.synchronize()
        graphs = []
        for i, p in enumerate(plans):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=side):
                p.execute(*views[i], out=outs[i % ring], stream=side)
            graphs.append(g)
        for g in graphs[:2]:
            g.replay()
        torch.cuda.synchronize()
        cur = torch.cuda.current_stream()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in graphs]
        t0 = time.perf_counter()
        for (a, z), g in zip(evs, graphs):
            a.record(cur)
            g.replay()
            z.record(cur)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lat = np.array([a.elapsed_time(z) for a, z in evs])
        ints = sum(p.output_size for p in plans)
        rec[prec] = {"value": ints / wall, "unit": "integrals/s", "s_per_pass": wall,
                     "pct_fp64_peak": 100 * flops / wall / 1e12 / FP64_PEAK_TFLOPS,
                     "chunk_ms_p50": float(np.percentile(lat, 50)), "chunk_ms_p99": float(np.percentile(lat, 99))}
        # the first chunk, kept for the FP32-vs-FP64 comparison
        graphs[0].replay()
        torch.cuda.synchronize()
        check[prec] = (plans[0], outs[0][:plans[0].output_size].clone())
        if prec == "fp64":
            rec["fp64"]["oracle_max_rel_err_sampled"] = sampled_oracle_err(inputs.subset(b, range(chunk)), plans[0],
                                                                           check["fp64"][1], smallest=True)
        del graphs, outs
    rec["fp32_speedup_vs_fp64"] = rec["fp64"]["s_per_pass"] / rec["fp32"]["s_per_pass"]
    rec["fp32_max_abs_err_vs_fp64_first_chunk"] = float((check["fp32"][1] - check["fp64"][1]).abs().max())
    return rec


def class_errors(b, plan, ref, test, target=1e-10):
    """Per class (la lb|lc ld): largest |test - ref| over all its quartets, with
    ref the FP64 path (itself within 1e-12 of the oracle relative to each
    quartet's largest integral), and the largest |ref|."""
    import numpy as np
    import torch
    off = torch.from_numpy(plan.offsets()).cuda()
    keys = [tuple(int(x) for x in r) for r in b.lq]
    by_cls = {}
    for q, k in enumerate(keys):
        by_cls.setdefault(k, []).append(q)
    per = []
    for k, qs in sorted(by_cls.items()):
        size = int(np.prod([(l + 1) * (l + 2) // 2 for l in k]))
        ar = torch.arange(size, device="cuda")
        err = mag = 0.0
        step = max(1, (1 << 26) // size)
        for i in range(0, len(qs), step):
            idx = off[torch.tensor(qs[i:i + step], device="cuda")][:, None] + ar[None, :]
            r = ref[idx]
            err = max(err, float((test[idx] - r).abs().max()))
            mag = max(mag, float(r.abs().max()))
        per.append({"class": "(%d%d|%d%d)" % k, "quartets": len(qs), "max_abs_err": err, "max_abs_integral": mag})
    worst = max(p["max_abs_err"] for p in per)
    return {"max_abs_err": worst, "target_abs_err": target, "meets_target": worst <= target,
            "classes_within_target": sum(p["max_abs_err"] <= target for p in per), "classes": len(per),
            "error_reference": "FP64 path on the same inputs (all quartets)",
            "worst_classes": sorted(per, key=lambda p: -p["max_abs_err"])[:5],
            "per_class_max_abs_err": {p["class"]: p["max_abs_err"] for p in per}}


def parity_sample(wl, b, out, n=2):
    import numpy as np
    import oracle
    from paper_2307_03452_amd import inputs
    idx = [0, b.nq - 1][:n]
    s = inputs.subset(b, idx)
    o = oracle.eri_md4(wl["ls"], s.centers, s.exps, s.coefs, s.nprim)
    g = out[idx].cpu().numpy()
    return max(float(np.abs(g[i] - o[i]).max() / np.abs(o[i]).max()) for i in range(len(idx)))


def cpu_baseline(wl, b, budget_s=12.0):
    """The oracle (as it stands) on the host cores, on the first quartets of the
    same workload, grown in chunks until about budget_s of CPU work."""
    import oracle
    from paper_2307_03452_amd import inputs, metrics
    threads = oracle.max_threads()
    done, t_tot = 0, 0.0
    chunk = max(threads, 1)
    while t_tot < budget_s and done < b.nq:
        idx = list(range(done, min(b.nq, done + chunk)))
        s = inputs.subset(b, idx)
        t0 = time.perf_counter()
        oracle.eri_md4(wl["ls"], s.centers, s.exps, s.coefs, s.nprim, nthreads=threads)
        t_tot += time.perf_counter() - t0
        done += len(idx)
        if t_tot < budget_s / 8:
            chunk *= 2
    ints = done * metrics.integrals_per_quartet(*wl["ls"])
    return {"value": ints / t_tot, "unit": "integrals/s", "cores": threads, "kind": "oracle",
            "sample": f"first {done} of the {b.nq} quartets of the same workload, OpenMP over quartets, "
                      f"{t_tot:.1f} s"}


def calibrate_copy(mib, reps=3):
    """dst = src + 0.0 on float64 tensors of mib MiB: one elementwise kernel
    that reads and writes exactly mib MiB per call."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.add(src, 0.0, out=dst)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB x {reps}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="iiii_k1", choices=sorted(WORKLOADS))
    ap.add_argument("--secondary-steps", type=int, default=1,
                    help="timed steps of the contracted (ii|ii) K=5 batch reported beside the headline (0: skip)")
    ap.add_argument("--uneven-steps", type=int, default=1,
                    help="timed steps of the 20k-quartet mixed-class batch reported beside the headline (0: skip)")
    ap.add_argument("--mixed-steps", type=int, default=1,
                    help="timed steps of the mixed-batch with FP32 transforms, compared with FP64 (0: skip)")
    ap.add_argument("--stream-steps", type=int, default=1,
                    help="run the l=7 classes and the 50k-quartet serving stream (0: skip)")
    ap.add_argument("--solid-steps", type=int, default=3,
                    help="timed calls of each solid-harmonic (ii|ii) batch (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-headline", action="store_true",
                    help="time the headline workload only (every other leg and the CPU baseline off), "
                         "e.g. for a profiler run whose dispatches must all belong to one workload")
    ap.add_argument("--legs", default=None,
                    help="comma list of the legs to run beside the headline (secondary, uneven, mixed, l7, stream, "
                         "low_l, pairs, gggg, solid, coulomb, exchange); default: all, unless --only-headline")
    ap.add_argument("--calibrate-copy", type=int, metavar="MIB", default=0,
                    help="instead of benchmarking, run a plain device copy (dst = src + 0) of MIB MiB of "
                         "float64 three times: the known-size kernel whose FETCH_SIZE/WRITE_SIZE counters "
                         "calibrate the integral kernel's")
    args = ap.parse_args()
    if args.calibrate_copy > 0:
        calibrate_copy(args.calibrate_copy)
        return
    if args.only_headline:
        args.secondary_steps = args.uneven_steps = args.mixed_steps = args.stream_steps = args.solid_steps = 0
        args.no_cpu_baseline = True
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (quartets would shard across GPUs "
              "with no communication). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    from paper_2307_03452_amd import metrics
    wl = WORKLOADS[args.workload]
    b = make_batch(wl)
    ls = wl["ls"]
    out, wall, launch_ms = time_gpu(wl, b, args.steps, args.warmup)
    ms_step = wall * 1e3 / args.steps
    ints = b.nq * metrics.integrals_per_quartet(*ls)
    kb = wl["K"] * wl["K"]
    flops = b.nq * metrics.md4_flops(*ls, kb, kb)
    avg_launch_s = sum(launch_ms) / len(launch_ms) / 1e3
    achieved = flops / avg_launch_s / 1e12
    rec = {
        "metric": METRIC,
        "value": ints / (wall / args.steps),
        "unit": "integrals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "quartets": b.nq, "K_per_shell": wl["K"],
                   "integrals_per_step": ints, "md4_flops_per_step": flops},
        "pct_fp64_peak": 100.0 * achieved / FP64_PEAK_TFLOPS,
        "md4_tflops": achieved,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic_from_profiles(args.workload),
                     "kernel": KERNEL, "avg_launch_ms": avg_launch_s * 1e3,
                     "algorithmic_unit": "MD4 matrix FLOPs per quartet x quartets per launch"},
    }
    rec["parity_max_rel_err"] = parity_sample(wl, b, out)
    legs = {"secondary": args.secondary_steps > 0, "uneven": args.uneven_steps > 0, "mixed": args.mixed_steps > 0,
            "l7": args.stream_steps > 0, "stream": args.stream_steps > 0, "low_l": args.stream_steps > 0,
            "pairs": args.stream_steps > 0, "gggg": args.stream_steps > 0, "solid": args.solid_steps > 0,
            "coulomb": args.solid_steps > 0, "exchange": args.solid_steps > 0}
    if args.legs is not None:
        chosen = {x for x in args.legs.split(",") if x}
        unknown = chosen - set(legs)
        if unknown:
            sys.exit(f"unknown legs: {sorted(unknown)}")
        legs = {k: k in chosen for k in legs}
    if args.workload != "iiii_k1":
        legs = {k: False for k in legs}
    reps = max(1, args.solid_steps)
    if legs["secondary"]:
        wl5 = WORKLOADS["iiii_k5"]
        b5 = make_batch(wl5)
        nsec = max(1, args.secondary_steps)
        _, wall5, lm5 = time_gpu(wl5, b5, nsec, 1)
        f5 = b5.nq * metrics.md4_flops(*ls, 25, 25)
        s5 = sum(lm5) / len(lm5) / 1e3
        rec["secondary"] = {"workload": wl5["desc"], "value": ints / (wall5 / nsec),
                            "unit": "integrals/s", "ms_per_step": wall5 * 1e3 / nsec,
                            "md4_tflops": f5 / s5 / 1e12, "pct_fp64_peak": 100 * f5 / s5 / 1e12 / FP64_PEAK_TFLOPS}
    if legs["uneven"] or legs["mixed"]:
        rec["uneven"], mixed = time_uneven(max(1, args.uneven_steps), 1,
                                           mixed_steps=max(1, args.mixed_steps) if legs["mixed"] else 0)
        if mixed is not None:
            rec["mixed_precision"] = mixed
    if legs["l7"]:
        rec["l7_classes"] = time_classes_l7()
    if legs["stream"]:
        rec["stream"] = time_stream()
    if legs["low_l"]:
        rec["low_l"] = time_low_l()
    if legs["pairs"]:
        rec["pairs"] = time_pairs()
    if legs["gggg"]:
        rec["gggg_k1"] = time_gggg()
    if legs["solid"]:
        rec["solid"] = time_solid(reps)
    if legs["coulomb"]:
        rec["coulomb"] = time_coulomb(reps)
    if legs["exchange"]:
        rec["exchange"] = time_exchange(reps)
    if not args.no_cpu_baseline:
        cb = cpu_baseline(wl, b)
        rec["cpu_baseline"] = cb
        rec["gpu_over_cpu"] = rec["value"] / cb["value"]
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
