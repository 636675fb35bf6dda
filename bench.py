#!/usr/bin/env python
"""Benchmark of the 4-centre MD path on one MI355X.

Workload (the l-class batches the metric is quoted on): [dd|dd], [ff|ff] and
[gg|gg] at K=1 and K=3 primitives per shell, each 256 bra x 256 ket shell
pairs (65,536 quartets), centres uniform in a 20-bohr cube, exponents
log-uniform in [0.05, 500], coefficients uniform in [0.1, 1]; pairs are
admitted by Schwarz screening (Q_ij Q_max >= 1e-12) from seeded candidates.
One step = the six class batches, each including its pair data and transform
matrices.  Inputs are resident in HBM before timing starts.

The backward/forward ratio is the time of the exchange-energy gradient
(dE/dR, E = tr(D K)) over the time of the K build itself, both on a synthetic
cluster (see inputs.cluster; --cluster-atoms sets its size).

Prints one JSON line (rank 0) with per-class rates, the roofline of the
dominant kernel (its launches timed by HIP events on the launch stream) and
the CPU oracle's rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

CLASSES = [(2, 1), (3, 1), (4, 1), (2, 3), (3, 3), (4, 3)]  # (l, K per shell)
NAMES = {2: "dd", 3: "ff", 4: "gg", 5: "hh", 6: "ii"}
NPAIR = 256
TAU = 1e-12


# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE (x2) and
# WRITE_SIZE (x1) counters (profiles/eri4_ggK3_hbm_counters.md), valid only for
# the kernel sources they were taken with.
TRAFFIC = {"kernel": "eri4_kernel [gg|gg] K=3", "bytes": 1.1302e11,
           "sources": {"eri4.hip": "03af330b91b2ba0e", "device_common.h": "1d6737b5b2d84adb",
                       "internal.h": "1f28521e37d5a89b"}}


def measured_traffic(kernel):
    import hashlib
    if kernel != TRAFFIC["kernel"]:
        return None
    for name, h in TRAFFIC["sources"].items():
        with open(os.path.join(ROOT, "paper_2405_01834_amd", "csrc", name), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest()[:16] != h:
                return None
    return TRAFFIC["bytes"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_batch(ctx, l, K, seed=1, npair=NPAIR):
    """Schwarz-admitted bra and ket pair lists of class (ll|ll) with K primitives per shell."""
    from paper_2405_01834_amd import inputs
    ncand = 4 * npair
    while True:
        ss = np.random.SeedSequence([seed, l, K, ncand])
        sh, cand = inputs.class_pairs(int(ss.generate_state(1)[0]), l, l, K, ncand)
        basis = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
        Q = ctx.schwarz(basis, cand).cpu().numpy()
        keep = np.nonzero(Q * Q.max() >= TAU)[0]
        if len(keep) >= 2 * npair:
            bra = cand[keep[:npair]]
            ket = cand[keep[npair:2 * npair]]
            return sh, basis, bra, ket, len(keep) / len(cand)
        basis.close()
        ncand *= 2


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(batches, outs, wall_per_class=2.5, pp_batch=None):
    """The oracle on a bounded sample of every class batch (all host threads,
    then one thread on a smaller sample); the sample's integrals are also
    compared element by element with the GPU output of the timed step.  The
    [pp|pp] 512-quartet batch is computed whole and compared the same way."""
    import oracle
    nthr = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
    total_eris, total_time, total_time1, parts = 0.0, 0.0, 0.0, []
    checked, worst, bad = 0, 0.0, 0
    for (l, K), (sh, _, bra, ket, _) in batches.items():
        ob = oracle.Basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, 1)
        nq_full = len(bra) * len(ket)
        n0 = min(nthr, len(ket))
        t = time.perf_counter()
        oracle.eri4(ob, bra[:1], ket[:n0], nthreads=nthr)
        t0 = max(time.perf_counter() - t, 1e-6)
        n = int(min(nq_full, max(n0, n0 * wall_per_class / t0)))
        nb = max(1, min(len(bra), n // len(ket)))
        nk = len(ket) if nb > 1 else max(1, min(len(ket), n))
        t = time.perf_counter()
        ref = oracle.eri4(ob, bra[:nb], ket[:nk], nthreads=nthr)
        dt = time.perf_counter() - t
        rate = nb * nk / dt
        # one thread on about a tenth of that sample
        n1 = max(1, min(nk, (nb * nk) // (10 * max(1, nb)) or 1))
        t = time.perf_counter()
        oracle.eri4(ob, bra[:1], ket[:n1], nthreads=1)
        rate1 = n1 / max(time.perf_counter() - t, 1e-9)
        nab = (2 * l + 1) ** 2
        got = outs[(l, K)].view(len(ket), nab, nab, len(bra)).permute(3, 2, 1, 0)[:nb, :, :, :nk].cpu().numpy()
        err = np.abs(got - ref)
        bad += int(np.sum(err > 1e-14 + 1e-12 * np.abs(ref)))
        checked += ref.size
        worst = max(worst, float(np.max(err / (1e-14 + 1e-12 * np.abs(ref)))))
        nb4 = nab * nab
        total_eris += nq_full * nb4
        total_time += nq_full / rate
        total_time1 += nq_full / rate1
        parts.append(f"{NAMES[l]}K{K}:{nb * nk}q")
        log(f"cpu oracle [{NAMES[l]}|{NAMES[l]}] K={K}: {nb * nk} quartets in {dt:.2f}s -> {rate:.1f} quartets/s "
            f"({rate1:.1f} on one thread); parity vs GPU: {int(np.sum(err > 1e-14 + 1e-12 * np.abs(ref)))} of "
            f"{ref.size} outside 1e-12/1e-14")
    pp = None
    if pp_batch is not None:
        sh, bra, ket, out = pp_batch
        ob = oracle.Basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, 1)
        t = time.perf_counter()
        ref = oracle.eri4(ob, bra, ket, nthreads=nthr)
        dt = time.perf_counter() - t
        got = out.view(len(ket), 9, 9, len(bra)).permute(3, 2, 1, 0).cpu().numpy()
        err = np.abs(got - ref)
        nbad = int(np.sum(err > 1e-14 + 1e-12 * np.abs(ref)))
        bad += nbad
        checked += ref.size
        worst = max(worst, float(np.max(err / (1e-14 + 1e-12 * np.abs(ref)))))
        pp = {"ms": dt * 1e3, "eris_per_s": ref.size / dt, "elements": ref.size, "outside_tolerance": nbad}
        log(f"cpu oracle [pp|pp] K=1: {len(bra) * len(ket)} quartets in {dt * 1e3:.1f} ms; parity vs GPU: {nbad} of "
            f"{ref.size} outside 1e-12/1e-14")
    return {"value": total_eris / total_time, "unit": "ERI/s", "cores": nthr, "kind": "oracle", "pp_small": pp,
            "single_core_value": total_eris / total_time1, "cpu_model": cpu_model(),
            "sample": "oracle FP64 on the first " + ", ".join(parts) +
                      " quartets of each class batch (single core: about a tenth of each); full-step time "
                      "extrapolated per class",
            "parity": {"elements": checked, "outside_tolerance": bad, "worst_err_over_tol": worst,
                       "tolerance": "|gpu - oracle| <= 1e-14 + 1e-12 |oracle|, GPU output of the last timed step"}}


def mixed_precision(ctx, steps):
    """[gg|gg], [hh|hh], [ii|ii], K=1, 128 x 128 Schwarz-admitted pairs (16,384
    quartets) each: FP64 against the split-precision bra transform with 5, 6
    and 7 slices; error per shellset (max |dV| - 1e-14) / max |V| against the
    FP64 result (max and RMS over shellsets)."""
    import torch
    from paper_2405_01834_amd import model
    from paper_2405_01834_amd.mderi import SPLIT_BF16
    out = {}
    for l in (4, 5, 6):
        sh, basis, bra, ket, frac = make_batch(ctx, l, 1, seed=4, npair=128)
        n = len(bra) * len(ket) * (2 * l + 1) ** 4
        ref = torch.empty(n, dtype=torch.float64, device="cuda")
        tmp = torch.empty(n, dtype=torch.float64, device="cuda")
        flops = len(bra) * len(ket) * model.eri4_flops(l, l, l, l, 1, 1)

        def timed(buf, **kw):
            ctx.eri4(basis, bra, ket, out=buf, **kw)  # warm-up (pair data, caches)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                ctx.eri4(basis, bra, ket, out=buf, **kw)
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / steps

        t64 = timed(ref)
        Vr = ref.view(len(ket), (2 * l + 1) ** 2, (2 * l + 1) ** 2, len(bra))
        mref = Vr.abs().amax(dim=(1, 2))
        name = f"[{NAMES[l]}|{NAMES[l]}] K=1"
        rec = {"fp64_ms": t64, "fp64_frac_peak": flops / (t64 * 1e-3) / 1e12 / model.FP64_PEAK_TFLOPS,
               "quartets": len(bra) * len(ket)}
        for S in (5, 6, 7):
            ts = timed(tmp, precision=SPLIT_BF16, slices=S)
            Vs = tmp.view_as(Vr)
            d = (Vs - Vr).abs().amax(dim=(1, 2))
            e = torch.clamp(d - 1e-14, min=0.0) / torch.clamp(mref, min=1e-300)
            rec[f"S{S}"] = {"ms": ts, "speedup": t64 / ts, "err_max": float(e.max()),
                            "err_rms": float(torch.sqrt((e * e).mean()))}
            log(f"{name}: FP64 {t64:.2f} ms; split S={S} {ts:.2f} ms (x{t64 / ts:.2f}), per-shellset error "
                f"max {float(e.max()):.2e} rms {float(torch.sqrt((e * e).mean())):.2e}")
        out[name] = rec
        basis.close()
        del ref, tmp, Vr
        torch.cuda.empty_cache()
    return {"classes": out,
            "workload": "[gg|gg],[hh|hh],[ii|ii] K=1, 128x128 Schwarz-admitted pairs each; error vs the FP64 "
                        "result per shellset, (max|dV| - 1e-14)/max|V|"}


def eri3_task_list(ctx, steps, flags):
    """512 mixed primary pairs x 512 auxiliary shells (262,144 triplets) in one
    task-list call; the first call builds, tunes and captures the plan."""
    import torch
    from paper_2405_01834_amd import inputs, model
    from paper_2405_01834_amd.mderi import FLAG_AUTOTUNE, FLAG_GRAPH
    prim, aux, pairs, auxidx = inputs.eri3_batch(3)
    b = ctx.basis(prim.l, prim.nprim, prim.exps, prim.coefs, prim.centers)
    a = ctx.basis(aux.l, aux.nprim, aux.exps, aux.coefs, aux.centers)
    fl = {"graph+autotune": FLAG_GRAPH | FLAG_AUTOTUNE, "graph": FLAG_GRAPH, "plain": 0}[flags]
    t = time.perf_counter()
    B = ctx.eri3_batch(b, a, pairs, auxidx, flags=fl)
    out = B.t().view(-1)
    torch.cuda.synchronize()
    first = time.perf_counter() - t
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        ctx.eri3_batch(b, a, pairs, auxidx, flags=fl, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    flops = 0.0
    for i, (p0, p1) in enumerate(pairs):
        kb = int(prim.nprim[p0] * prim.nprim[p1])
        for k in auxidx:
            flops += model.eri3_flops(int(prim.l[p0]), int(prim.l[p1]), int(aux.l[k]), kb, 1)
    ntrip = len(pairs) * len(auxidx)
    neri = B.shape[0] * B.shape[1]
    log(f"eri3 task list ({flags}): {ntrip} triplets, {neri} ERIs, {ms:.3f} ms per call "
        f"({ntrip / (ms * 1e-3):.3e} triplets/s, {flops / (ms * 1e-3) / 1e12:.2f} TFLOP/s); first call {first:.2f} s")
    return {"ms": ms, "triplets": ntrip, "eris": neri, "triplets_per_s": ntrip / (ms * 1e-3),
            "eris_per_s": neri / (ms * 1e-3), "model_tflops": flops / (ms * 1e-3) / 1e12,
            "frac_fp64_peak": flops / (ms * 1e-3) / 1e12 / model.FP64_PEAK_TFLOPS, "flags": flags,
            "first_call_s": first,
            "workload": "512 primary pairs (l_a, l_b in 0..3, K 1..5 per shell) x 512 auxiliary shells "
                        "(l_P in 0..6, K=1); 20-bohr cube, exponents log-U[0.05,500]; one mderi_eri3_batch call"}


def eri2_metric(ctx, steps):
    """The 2-centre Coulomb metric (P|Q) of the 512 auxiliary shells of the
    3-centre workload (l_P 0..6, K=1): every class batch (l_a | l_c), both
    triangles, timed as one step."""
    import torch
    from paper_2405_01834_amd import inputs, model
    _, aux, _, _ = inputs.eri3_batch(3)
    a = ctx.basis(aux.l, aux.nprim, aux.exps, aux.coefs, aux.centers)
    by_l = {l: np.flatnonzero(aux.l == l).astype(np.int32) for l in sorted(set(int(x) for x in aux.l))}
    outs = {}
    flops = 0.0
    for la, A in by_l.items():
        for lc, C in by_l.items():
            # flat outputs allocated once, so the timed calls allocate nothing
            outs[(la, lc)] = torch.empty(len(A) * (2 * la + 1) * (2 * lc + 1) * len(C), dtype=torch.float64,
                                         device="cuda")
            ctx.eri2(a, A, C, out=outs[(la, lc)])
            # the 3-centre model with a one-centre bra (l_b = 0)
            flops += len(A) * len(C) * model.eri3_flops(la, 0, lc, 1, 1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    gc.disable()  # host-bound loop: no cyclic-GC pause inside the timed region
    e0.record()
    for _ in range(steps):
        for (la, lc), V in outs.items():
            ctx.eri2(a, by_l[la], by_l[lc], out=V)
    e1.record()
    torch.cuda.synchronize()
    gc.enable()
    ms = e0.elapsed_time(e1) / steps
    nao = int(np.sum(2 * aux.l + 1))
    log(f"eri2 metric: {len(aux.l)} shells, {nao}x{nao} elements, {ms:.3f} ms ({nao * nao / (ms * 1e-3):.3e} "
        f"elements/s, {flops / (ms * 1e-3) / 1e12:.2f} TFLOP/s)")
    return {"ms": ms, "shells": int(len(aux.l)), "elements": nao * nao, "elements_per_s": nao * nao / (ms * 1e-3),
            "model_tflops": flops / (ms * 1e-3) / 1e12,
            "frac_fp64_peak": flops / (ms * 1e-3) / 1e12 / model.FP64_PEAK_TFLOPS, "class_batches": len(outs),
            "workload": "2-centre metric of the 512 auxiliary shells of the 3-centre workload (l 0..6, K=1, "
                        "20-bohr cube, exponents log-U[0.05,500]); all 49 class batches, both triangles"}


def high_l_aux(ctx, steps):
    """3-centre class batches with auxiliary shells beyond l = 6: 256 (dd)
    pairs (K=3 per shell) x 256 auxiliary shells of l = 7 and of l = 8 (K=1)."""
    import torch
    from paper_2405_01834_amd import inputs, model
    rng = np.random.default_rng(8)
    prim = inputs.random_shells(rng, [2] * 512, 3, 20.0, 0.05, 500.0)
    b = ctx.basis(prim.l, prim.nprim, prim.exps, prim.coefs, prim.centers)
    pairs = np.arange(512, dtype=np.int32).reshape(-1, 2)
    res = {}
    for lP in (7, 8):
        aux = inputs.random_shells(rng, [lP] * 256, 1, 20.0, 0.05, 500.0)
        a = ctx.basis(aux.l, aux.nprim, aux.exps, aux.coefs, aux.centers)
        idx = np.arange(256, dtype=np.int32)
        V = ctx.eri3(b, a, pairs, idx)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        flat = V.permute(3, 2, 1, 0).reshape(-1)
        e0.record()
        for _ in range(steps):
            ctx.eri3(b, a, pairs, idx, out=flat)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        flops = len(pairs) * len(idx) * model.eri3_flops(2, 2, lP, 9, 1)
        res[f"(dd|{lP})"] = {"ms": ms, "triplets_per_s": len(pairs) * len(idx) / (ms * 1e-3),
                             "model_tflops": flops / (ms * 1e-3) / 1e12,
                             "frac_fp64_peak": flops / (ms * 1e-3) / 1e12 / model.FP64_PEAK_TFLOPS}
        log(f"(dd|{lP}) K=3: {ms:.3f} ms ({flops / (ms * 1e-3) / 1e12:.2f} TFLOP/s)")
    res["workload"] = ("256 (dd) pairs, K=3 per shell, x 256 auxiliary shells of l = 7 and of l = 8 (K=1); 20-bohr "
                       "cube, exponents log-U[0.05,500]")
    return res


def dfj_leg(ctx, natom=12):
    """Density-fitted J and K on the cluster recipe with an even-tempered
    fitting set per atom (s12 p8 d6 f4 g3 h2, exponents geometric from 0.16 to
    twice the largest primary exponent for s, narrower ranges for higher l),
    against the 4-centre J and K of the quartet engine: time of one call each
    (after a warm-up), with the factors computed and with the factors the
    context kept, and the relative errors of tr(D J) and tr(D K)."""
    import torch
    from paper_2405_01834_amd import inputs
    sh, atom, pos, D = inputs.cluster(7, natom)
    b = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, atom=atom)
    ls, ex, cen = [], [], []
    for p in pos:
        for l, n, hi in ((0, 12, 4000.0), (1, 8, 500.0), (2, 6, 100.0), (3, 4, 40.0), (4, 3, 25.0), (5, 2, 10.0)):
            for z in np.geomspace(0.16, hi, n):
                ls.append(l)
                ex.append(z)
                cen.append(p)
    a = ctx.basis(np.array(ls, np.int32), np.ones(len(ls), np.int32), np.array(ex), np.ones(len(ls)), np.array(cen))
    Dd = torch.tensor(D, device="cuda")
    bcen = torch.tensor(sh.centers, device="cuda")

    def timed(fn, cold):
        # cold: the basis is set to the same centres first, which drops the
        # factors the context kept, so (ab|P), the metric and its factor are
        # computed again; warm: the kept factors of the previous call
        if cold:
            b.set_centers(bcen)
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn(b, a, Dd)
        torch.cuda.synchronize()
        return out, time.perf_counter() - t

    ctx.dfj(b, a, Dd)
    ctx.dfk(b, a, Dd)
    Jdf, tdf = timed(ctx.dfj, True)
    _, tdf_warm = timed(ctx.dfj, False)
    Kdf, tdk = timed(ctx.dfk, True)
    _, tdk_warm = timed(ctx.dfk, False)
    J, K = ctx.jkbuild(b, Dd, tau=TAU)
    torch.cuda.synchronize()
    e, edf = float(torch.sum(Dd * J)), float(torch.sum(Dd * Jdf))
    ek, ekdf = float(torch.sum(Dd * K)), float(torch.sum(Dd * Kdf))
    nrow = int(sum((2 * sh.l[i] + 1) * (2 * sh.l[j] + 1) for i in range(sh.n) for j in range(i + 1)))
    nao, naux = b.nao(), a.nao()
    gemm_tflops = 4.0 * nao ** 3 * naux / tdk / 1e12  # the two GEMMs alone, over the whole call's time
    log(f"DF-J {natom} atoms: {naux} fitting AOs, {nrow} pair rows, {tdf * 1e3:.1f} ms; "
        f"tr(DJ) relative error {abs(edf - e) / abs(e):.2e}")
    # (the random rank-100 density couples every pair of atoms, and an
    # atom-centred fitting set does not span the cross-atom pair products that
    # tr(DK) weighs, so DF-K sits well below the 4-centre value; tr(DJ) is
    # dominated by near-diagonal products and fits to 1e-3)
    log(f"DF-K {natom} atoms: {tdk * 1e3:.1f} ms ({gemm_tflops:.1f} TFLOP/s of GEMM over the call); "
        f"tr(DK) relative error {abs(ekdf - ek) / abs(ek):.2e}")
    log(f"DF with the kept factors: J {tdf_warm * 1e3:.2f} ms, K {tdk_warm * 1e3:.2f} ms "
        f"({4.0 * nao ** 3 * naux / tdk_warm / 1e12:.1f} TFLOP/s of GEMM)")
    return {"ms": tdf * 1e3, "atoms": natom, "nao": nao, "fitting_aos": naux, "pair_rows": nrow,
            "triplets": int(sh.n * (sh.n + 1) // 2 * len(ls)), "energy_rel_err": abs(edf - e) / abs(e),
            "dfk_ms": tdk * 1e3, "dfk_energy_rel_err": abs(ekdf - ek) / abs(ek), "dfk_gemm_tflops": gemm_tflops,
            "warm_ms": tdf_warm * 1e3, "dfk_warm_ms": tdk_warm * 1e3,
            "dfk_warm_gemm_tflops": 4.0 * nao ** 3 * naux / tdk_warm / 1e12,
            "workload": "cluster recipe, %d atoms; fitting set per atom s12 p8 d6 f4 g3 h2 (K=1, even-tempered "
                        "from 0.16 to 4000/500/100/40/25/10); one mderi_dfj and one mderi_dfk call (all "
                        "canonical pairs, no screening) after a warm-up, each cold (factors computed: ms, "
                        "dfk_ms) and with the factors the context kept from the previous call (warm_ms, "
                        "dfk_warm_ms)" % natom}


def count_quartets(ctx, basis, sh):
    """Symmetry-unique quartets of the K build and ordered visits of the
    gradient that pass the screening (Q_ij Q_max >= tau for pairs, Q_ij Q_kl
    >= tau for quartets), from the GPU's Schwarz factors of all canonical pairs."""
    import torch
    l = sh.l
    i, j = np.nonzero((l[:, None] > l[None, :]) | ((l[:, None] == l[None, :]) &
                                                   (np.arange(sh.n)[:, None] >= np.arange(sh.n)[None, :])))
    pairs = np.stack([i, j], axis=1).astype(np.int32)
    Q = ctx.schwarz(basis, pairs).cpu().numpy()
    torch.cuda.synchronize()
    keep = Q * Q.max() >= TAU
    q = np.sort(Q[keep])
    ordered = int(np.sum(len(q) - np.searchsorted(q, TAU / q, side="left")))
    diag = int(np.sum(q * q >= TAU))
    return (ordered + diag) // 2, ordered, int(keep.sum())


def pp_small(ctx, reps=200):
    """[pp|pp] K=1, 512 shell quartets (16 bra x 32 ket pairs, centres in a
    10-bohr cube, exponents log-U[0.1,100], no screening): the launch-bound
    end of the class table.  One call = the pair data of both sides (one
    launch each) + the fused kernel; the stream time per call from events
    around `reps` back-to-back calls, the fused kernel's own time from the
    library's events (a second pass), the host time per call from the wall
    clock."""
    import torch
    from paper_2405_01834_amd import inputs, model
    sh, bra, ket = inputs.pp_quartets(0)
    basis = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers)
    out = torch.empty(len(bra) * len(ket) * 81, dtype=torch.float64, device="cuda")
    for _ in range(5):
        ctx.eri4(basis, bra, ket, out=out)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    gc.disable()  # host-bound loop: no cyclic-GC pause inside the timed region
    t = time.perf_counter()
    start.record()
    for _ in range(reps):
        ctx.eri4(basis, bra, ket, out=out)
    stop.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t) / reps
    gc.enable()
    # the fused kernel's own time in a second pass: the library's events
    # around each launch would otherwise add to the host and stream times
    ctx.kernel_times()
    ctx.kernel_timing(True)
    for _ in range(reps):
        ctx.eri4(basis, bra, ket, out=out)
    torch.cuda.synchronize()
    ctx.kernel_timing(False)
    kern = float(ctx.kernel_times().mean())
    ms = start.elapsed_time(stop) / reps
    nq = len(bra) * len(ket)
    eris = nq * model.eri4_outputs(1, 1, 1, 1)
    flops = nq * model.eri4_flops(1, 1, 1, 1, 1, 1)
    log(f"[pp|pp] K=1, {nq} quartets: {ms * 1e3:.1f} us per call on the stream ({kern * 1e3:.1f} us fused kernel, "
        f"{wall * 1e6:.1f} us host), {eris / (ms * 1e-3):.3e} ERI/s")
    return {"quartets": nq, "ms": ms, "kernel_ms": kern, "host_ms_per_call": wall * 1e3,
            "eris_per_s": eris / (ms * 1e-3), "kernel_eris_per_s": eris / (kern * 1e-3),
            "model_tflops": flops / (ms * 1e-3) / 1e12,
            "frac_fp64_peak": flops / (ms * 1e-3) / 1e12 / model.FP64_PEAK_TFLOPS,
            "workload": "[pp|pp] K=1, 16 x 32 pairs (512 quartets), 10-bohr cube, exponents log-U[0.1,100], "
                        "seed 0, %d back-to-back calls" % reps}, (sh, bra, ket, out)


def backward_forward(ctx, natom, warm_atoms=12):
    """Exchange-gradient time over K-build time on the synthetic cluster
    (inputs.cluster): both calls first run on a small cluster of the same
    recipe (same kernels), then once each on the full cluster; wall clock
    around call + synchronisation (host pair selection included)."""
    import torch
    from paper_2405_01834_amd import inputs
    sw, aw, _, Dw = inputs.cluster(7, warm_atoms)
    bw = ctx.basis(sw.l, sw.nprim, sw.exps, sw.coefs, sw.centers, atom=aw)
    Dwd = torch.tensor(Dw, device="cuda")
    ctx.kbuild(bw, Dwd, tau=TAU)
    ctx.jkbuild(bw, Dwd, tau=TAU)
    ctx.jkbuild(bw, Dwd, tau=TAU, deterministic=True)
    ctx.kbuild_grad(bw, Dwd, warm_atoms, tau=TAU)
    torch.cuda.synchronize()
    bw.close()
    sh, atom, pos, D = inputs.cluster(7, natom)
    basis = ctx.basis(sh.l, sh.nprim, sh.exps, sh.coefs, sh.centers, atom=atom)
    ctx.progress(natom >= 100)  # calls of minutes: one line per finished launch group
    Dd = torch.tensor(D, device="cuda")
    nq, nord, npair = count_quartets(ctx, basis, sh)
    log(f"cluster {natom} atoms, {sh.n} shells, {basis.nao()} AOs: {npair} significant pairs, {nq:.4g} unique "
        f"quartets, {nord:.4g} ordered")

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t, r

    tf, K = timed(lambda: ctx.kbuild(basis, Dd, tau=TAU))
    log(f"  K build {tf:.2f} s ({nq / tf:.3e} quartets/s)")
    tb, g = timed(lambda: ctx.kbuild_grad(basis, Dd, natom, tau=TAU))
    log(f"  gradient {tb:.2f} s ({nq / tb:.3e} quartets/s), ratio {tb / tf:.2f}")
    tjk, (Ja, Ka) = timed(lambda: ctx.jkbuild(basis, Dd, tau=TAU))
    log(f"  J+K build {tjk:.2f} s")
    tdet, (Jd, Kd) = timed(lambda: ctx.jkbuild(basis, Dd, tau=TAU, deterministic=True))
    det_dev = max(float((Kd - Ka).abs().max() / Ka.abs().max()), float((Jd - Ja).abs().max() / Ja.abs().max()))
    log(f"  J+K build, deterministic {tdet:.2f} s, max |d| / max |ref| from the atomic build {det_dev:.1e}")
    ctx.progress(False)
    gs = g.cpu().numpy()
    return {"ratio": tb / tf, "forward_ms": tf * 1e3, "backward_ms": tb * 1e3, "jk_build_ms": tjk * 1e3,
            "jk_build_deterministic_ms": tdet * 1e3, "deterministic_vs_atomic": det_dev,
            "atoms": natom, "shells": int(sh.n), "nao": basis.nao(), "significant_pairs": npair,
            "kbuild_quartets": nq, "ordered_quartets": nord, "kbuild_quartets_per_s": nq / tf,
            "gradient_quartets_per_s": nq / tb,
            "translational_residual": float(np.max(np.abs(gs.sum(axis=0))) / np.max(np.abs(gs))),
            "workload": "synthetic cluster, per atom s4 p3 d2 f1 g1 (K=1, exponents geometric 0.08-2000), "
                        "atoms >= 2 bohr apart in a 30-bohr box at 150 atoms, rank-100 PSD density, Schwarz "
                        "1e-12; forward = K build, backward = dE/dR of tr(DK); one call each after a warm-up "
                        "on %d atoms" % warm_atoms}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-wall", type=float, default=2.5, help="oracle wall seconds per class")
    ap.add_argument("--classes", default="", help="subset, e.g. 4:3,2:1 (l:K)")
    ap.add_argument("--no-split", action="store_true", help="skip the split-precision comparison")
    ap.add_argument("--no-tune", action="store_true", help="skip the per-class autotuning of the 4-centre batches")
    ap.add_argument("--eri3", default="graph+autotune", choices=["graph+autotune", "graph", "plain", "off"],
                    help="mode of the 3-centre task-list measurement")
    ap.add_argument("--cluster-atoms", type=int, default=40,
                    help="atoms of the cluster for the backward/forward ratio (0 = skip); the full recipe size "
                         "is 150 atoms, minutes per call, so the default run takes 40")
    ap.add_argument("--cluster-only", action="store_true",
                    help="only the backward/forward leg (e.g. --cluster-only --cluster-atoms 150)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 2 GiB device-to-device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        a = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("copied 2 GiB")
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the integral batches are independent per GPU and this build "
              "has no multi-GPU path; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2405_01834_amd import Context, model

    if args.cluster_only:
        ctx = Context(0)
        bf = backward_forward(ctx, args.cluster_atoms)
        rec = {"metric": "backward/forward time ratio (exchange gradient / K build)", "value": bf["ratio"],
               "unit": "ratio", "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": bf["forward_ms"] + bf["backward_ms"],
               "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
               "config": {"workload": f"synthetic cluster, {args.cluster_atoms} atoms"}, "backward_forward": bf}
        print(json.dumps(rec), flush=True)
        return

    classes = CLASSES
    if args.classes:
        classes = [tuple(int(x) for x in c.split(":")) for c in args.classes.split(",")]
    ctx = Context(0)
    batches = {}
    for l, K in classes:
        batches[(l, K)] = make_batch(ctx, l, K)
        log(f"[{NAMES[l]}|{NAMES[l]}] K={K}: admitted fraction {batches[(l, K)][4]:.2f}")
    outs = {}
    for (l, K), (sh, basis, bra, ket, _) in batches.items():
        n = len(bra) * len(ket) * (2 * l + 1) ** 4
        outs[(l, K)] = torch.empty(n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    def step(events=None):
        for i, ((l, K), (sh, basis, bra, ket, _)) in enumerate(batches.items()):
            if events is not None:
                events[i][0].record()
            ctx.eri4(basis, bra, ket, out=outs[(l, K)])
            if events is not None:
                events[i][1].record()

    if not args.no_tune:
        # autotune: the first call of each class times its work-split variants
        from paper_2405_01834_amd.mderi import FLAG_AUTOTUNE
        t = time.perf_counter()
        for (l, K), (sh, basis, bra, ket, _) in batches.items():
            ctx.eri4(basis, bra, ket, out=outs[(l, K)], flags=FLAG_AUTOTUNE)
        torch.cuda.synchronize()
        log(f"autotune: {time.perf_counter() - t:.1f} s")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in batches]
          for _ in range(args.steps)]
    per = {k: 0.0 for k in batches}
    ctx.kernel_times()
    ctx.kernel_timing(True)
    t0 = time.perf_counter()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for s in range(args.steps):
        step(ev[s])
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.kernel_timing(False)
    kt = ctx.kernel_times().reshape(args.steps, len(batches))
    kern = {k: float(kt[:, i].mean()) for i, k in enumerate(batches)}
    total_ms = start.elapsed_time(stop)
    for s in range(args.steps):
        for i, k in enumerate(batches):
            per[k] += ev[s][i][0].elapsed_time(ev[s][i][1]) / args.steps

    eris_step = 0
    per_class = {}
    dom, dom_flops, dom_ms = None, 0.0, 0.0
    for (l, K), (sh, basis, bra, ket, frac) in batches.items():
        nq = len(bra) * len(ket)
        eris = nq * model.eri4_outputs(l, l, l, l)
        eris_step += eris
        flops = nq * model.eri4_flops(l, l, l, l, K * K, K * K)
        ms = per[(l, K)]
        name = f"[{NAMES[l]}|{NAMES[l]}] K={K}"
        per_class[name] = {"ms": round(ms, 4), "kernel_ms": round(kern[(l, K)], 4), "quartets": nq,
                           "shellsets_per_s": nq / (ms * 1e-3),
                           "eris_per_s": eris / (ms * 1e-3), "model_tflops": flops / (ms * 1e-3) / 1e12,
                           "frac_fp64_peak": flops / (ms * 1e-3) / 1e12 / model.FP64_PEAK_TFLOPS}
        if flops > dom_flops:
            dom, dom_flops, dom_ms = name, flops, kern[(l, K)]
        log(f"{name}: {ms:.3f} ms  {per_class[name]['shellsets_per_s']:.3e} shellsets/s  "
            f"{per_class[name]['model_tflops']:.2f} TFLOP/s ({100 * per_class[name]['frac_fp64_peak']:.1f}% FP64 peak)")
    ms_step = total_ms / args.steps
    value = eris_step / (ms_step * 1e-3)
    achieved = dom_flops / (dom_ms * 1e-3) / 1e12
    rec = {
        "metric": "shell-quartet ERIs/s and % FP64 peak per l-class; backward/forward time ratio",
        "value": value, "unit": "ERI/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "4-centre class batches [dd|dd],[ff|ff],[gg|gg] x K=1,3 per shell; 256x256 "
                               "Schwarz-admitted pairs (65,536 quartets) each; 20-bohr cube, exponents "
                               "log-U[0.05,500], coefficients U[0.1,1]", "quartets_per_class": NPAIR * NPAIR,
                   "classes": [f"{NAMES[l]}K{K}" for l, K in classes], "autotuned": not args.no_tune},
        "per_class": per_class,
        "roofline": {"bound": "mfma", "kernel": f"eri4_kernel {dom}", "kernel_ms": dom_ms, "achieved": achieved,
                     "peak": model.FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / model.FP64_PEAK_TFLOPS,
                     "traffic": measured_traffic(f"eri4_kernel {dom}"), "traffic_unit": "B"},
        "wall_s": wall,
    }
    rec["pp_small"], pp_batch = pp_small(ctx)
    if not args.no_split:
        rec["mixed_precision"] = mixed_precision(ctx, max(args.steps, 2))
    if args.eri3 != "off":
        rec["eri3_batch"] = eri3_task_list(ctx, max(args.steps, 3), args.eri3)
        rec["eri2_metric"] = eri2_metric(ctx, max(args.steps, 3))
        rec["high_l_aux"] = high_l_aux(ctx, max(args.steps, 3))
        rec["dfj"] = dfj_leg(ctx)
    if args.cluster_atoms > 0:
        rec["backward_forward"] = backward_forward(ctx, args.cluster_atoms)
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(batches, outs, args.cpu_wall, pp_batch)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
