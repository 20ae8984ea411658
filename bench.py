"""Benchmark: screened ERI quartets/s and Fock-build time on one MI355X.

Workload: 64 waters on a jittered 4^3 lattice (seed 1), s/p/d synthetic
basis, 640 shells, 1216 basis functions, Schwarz threshold 1e-10 (a seeded
stand-in for the paper's graphene bilayers in 6-31G(d), section 5.2).
A step is one direct Fock build F = H + 2J - K from the converged FP64 SCF
density (density preparation, all 21 quartet-class kernels, assembly), with
the density and all data resident in HBM.  The FP64 build is the headline;
the mixed-precision build (FP32 for quartets with Q_ab Q_cd max|D| < 1e-7) is
timed the same way and reported with its error against the FP64 build.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]

Prints one JSON line.
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

FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 flop/clk
SETUP_FLOPS = 20            # per primitive quartet: p+q, 1/(p+q), rho, P-Q, T, prefactor, W-P, W-Q
BOYS_FLOPS_TAYLOR = 3 * 7 + 4  # 8-term Taylor at the nearest grid point
# sources that determine the class kernels and their launch plans: counter
# readings stored under profiles/ apply only while these are unchanged
KERNEL_SOURCES = ["paper_1708_00033_amd/csrc/eri_impl.h", "paper_1708_00033_amd/csrc/hfx_internal.h",
                  "paper_1708_00033_amd/csrc/gen_eri.py", "paper_1708_00033_amd/csrc/hfx_api.cpp",
                  "paper_1708_00033_amd/csrc/eri_dispatch.hip"]


def class_flop_model():
    """Algorithmic flops of each class: per primitive quartet (setup, Boys
    with downward recursion, vertical recurrence) and per quartet
    (horizontal recurrences, contraction sums, 6 updates x 2 flops per
    integral for the digestion of eq. 2)."""
    sys.path.insert(0, os.path.join(ROOT, "paper_1708_00033_amd", "csrc"))
    import gen_eri
    out = []
    for (B, K) in gen_eri.CLASSES:
        la, lb = gen_eri.PAIR_CLASSES[B]
        lc, ld = gen_eri.PAIR_CLASSES[K]
        g = gen_eri.ClassGen(la, lb, lc, ld)
        g.emit("x")
        L = la + lb + lc + ld
        nint = gen_eri.ncart(la) * gen_eri.ncart(lb) * gen_eri.ncart(lc) * gen_eri.ncart(ld)
        es, fs = g.targets()
        per_prim = SETUP_FLOPS + BOYS_FLOPS_TAYLOR + 3 * L + L + g.flops + len(es) * len(fs)
        per_quartet = g.hrr_flops + 12 * nint
        out.append((per_prim, per_quartet, nint))
    return out


def source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def host_cpu():
    """The host's processor as lscpu reports it, and the CPUs this process may use."""
    import subprocess
    kv = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            kv[k.strip()] = v.strip()
    except Exception:
        pass

    def num(k):
        try:
            return int(kv.get(k, ""))
        except ValueError:
            return None
    return {"model": kv.get("Model name"), "sockets": num("Socket(s)"), "cores_per_socket": num("Core(s) per socket"),
            "threads_per_core": num("Thread(s) per core"), "cpus_online": num("CPU(s)"),
            "cpus_usable": len(os.sched_getaffinity(0))}


_ONE_THREAD_SAMPLE = r"""
import json, sys, time
sys.path.insert(0, %r)
import numpy as np, oracle, workloads as W
m = W.cluster64_config()
D = np.load(%r)
B = oracle.Basis(m)
B.schwarz()
t0 = time.time()
_, _, st = B.jk(D, 1e-10, stride=%d, phase=0)
dt = time.time() - t0
print(json.dumps({"quartets": st[0], "seconds": dt, "threads": oracle.num_threads()}))
"""


def cpu_baseline(mol, D, target_s=15.0, one_thread_s=6.0):
    """The CPU oracle's 8-fold Fock build on a bounded sample of the same
    workload: every stride-th bra shell pair (all its kets), sized for about
    target_s seconds, with the OpenMP threads the process has; then a smaller
    sample on one thread (a child process with OMP_NUM_THREADS=1)."""
    import subprocess
    import tempfile
    import numpy as np
    import oracle
    B = oracle.Basis(mol)
    B.schwarz()
    nthreads = oracle.num_threads()
    # grow the sample (smaller stride) until it takes about target_s seconds
    stride = 20011
    while True:
        t0 = time.time()
        _, _, st2 = B.jk(D, 1e-10, stride=stride, phase=0)
        dt2 = time.time() - t0
        if dt2 >= 0.6 * target_s or stride == 1:
            break
        stride = max(1, int(stride * max(dt2, 0.05) / target_s))
    rate = st2[0] / dt2
    one = None
    with tempfile.TemporaryDirectory() as td:
        dpath = os.path.join(td, "D.npy")
        np.save(dpath, D)
        # one thread at the sample's per-thread rate: stride scaled to about one_thread_s seconds
        s1 = max(stride, int(stride * nthreads * dt2 / one_thread_s))
        env = dict(os.environ, OMP_NUM_THREADS="1")
        try:
            out = subprocess.run([sys.executable, "-c", _ONE_THREAD_SAMPLE % (ROOT, dpath, s1)], env=env,
                                 capture_output=True, text=True, timeout=300)
            r1 = json.loads(out.stdout.strip().splitlines()[-1])
            one = {"value": r1["quartets"] / r1["seconds"], "threads": r1["threads"], "quartets": r1["quartets"],
                   "seconds": round(r1["seconds"], 2), "stride": s1}
        except Exception as e:   # reported, not fatal: the multi-threaded sample is the baseline
            one = {"error": str(e)[:200]}
    return dict(value=rate, unit="quartets/s", cores=nthreads, kind="oracle",
                sample=f"bra shell pairs with index % {stride} == 0 (all their kets): {st2[0]} screened quartets, "
                       f"{st2[1]} integrals in {dt2:.1f} s, FP64 McMurchie-Davidson, OpenMP over bra pairs, "
                       f"{nthreads} threads",
                host=host_cpu(), one_thread=one, seconds=dt2)


def batched_bench(args, log):
    """256 independent clusters of 1-16 waters (sizes seeded), one batched
    build per step (one launch per quartet class and ket list for all of them)
    vs the same 256 molecules built one context at a time; FP64, mixed and a
    HIP-graph replay of the FP64 batched build.  Densities: per molecule an
    orthogonal projector onto nocc random directions (the screened quartet set,
    hence the FP64 work, does not depend on D)."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1708_00033_amd import hfx, autotune
    mols = W.cluster_batch(256, 2)
    t0 = time.time()
    bctx = hfx.Context(device=0).load_batch(mols)
    t_load = time.time() - t0
    nbf, nocc, off, tot = bctx.layout
    Dh = np.concatenate([W.random_orthonormal_density(int(n), int(o), 1000 + i).ravel()
                         for i, (n, o) in enumerate(zip(nbf, nocc))])
    dev = torch.device("cuda:0")
    D = torch.tensor(Dh, device=dev)
    F = torch.empty_like(D)
    stream = torch.cuda.Stream(dev)
    sp = stream.cuda_stream
    counts = bctx.class_counts()
    quartets = int(counts[:, 0].sum())
    with torch.cuda.stream(stream):
        tuning = autotune.autotune(bctx, D.data_ptr(), F.data_ptr(), sp, sync=stream.synchronize)

        def time_builds(fn, n):
            fn()
            stream.synchronize()
            t = time.perf_counter()
            for _ in range(n):
                fn()
            stream.synchronize()
            return (time.perf_counter() - t) / n

        def class_ms():
            bctx.kernel_timing(True)
            bctx.build_fock_dev(D.data_ptr(), F.data_ptr(), sp)
            stream.synchronize()
            ms, _ = bctx.kernel_times()
            bctx.kernel_timing(False)
            order = np.argsort(-ms)[:8]
            return {hfx.CLASS_NAMES[k]: round(float(ms[k]), 3) for k in order}

        bctx.configure(precision=hfx.HFX_PREC_FP64)
        t64 = time_builds(lambda: bctx.build_fock_dev(D.data_ptr(), F.data_ptr(), sp), args.steps)
        F64 = F.clone()
        cms64 = class_ms()
        bctx.graph_capture(D.data_ptr(), F.data_ptr(), sp)
        tg = time_builds(lambda: bctx.graph_launch(sp), args.steps)
        graph_err = (F - F64).abs().max().item()
        bctx.configure(precision=hfx.HFX_PREC_MIXED)
        ptab = autotune.autotune_precision(bctx, D.data_ptr(), F.data_ptr(), sp, sync=stream.synchronize)
        tmx = time_builds(lambda: bctx.build_fock_dev(D.data_ptr(), F.data_ptr(), sp), args.steps)
        mixed_err = (F - F64).abs().max().item()
        cmsmx = class_ms()
        stm = bctx.build_fock_dev(D.data_ptr(), F.data_ptr(), sp, stats=True)
        bctx.configure(precision=hfx.HFX_PREC_FP64)
        # the same molecules one context (and one set of launches) at a time
        ctxs = [hfx.Context(device=0).load(m) for m in mols]
        Ds = [D[int(o):int(o) + int(n) * int(n)] for o, n in zip(off, nbf)]
        Fs = [F[int(o):int(o) + int(n) * int(n)] for o, n in zip(off, nbf)]

        def one_by_one():
            for c, d, f in zip(ctxs, Ds, Fs):
                c.build_fock_dev(d.data_ptr(), f.data_ptr(), sp)
        tseq = time_builds(one_by_one, max(1, args.steps // 2))
        seq_err = (F - F64).abs().max().item()
        # SCF: all 256 in lockstep vs the first 32 one molecule at a time
        stream.synchronize()
        t = time.perf_counter()
        bres, _ = bctx.batch_scf()
        t_bscf = time.perf_counter() - t
        t = time.perf_counter()
        gres, _ = bctx.batch_scf(graph=1)   # each iteration's device work replayed from HIP graphs
        t_gscf = time.perf_counter() - t
        dEg = max(abs(a["energy"] - b["energy"]) for a, b in zip(gres, bres))
        t = time.perf_counter()
        sres = [c.scf() for c in ctxs[:32]]
        t_sscf32 = time.perf_counter() - t
        dE = max(abs(b["energy"] - r["energy"]) for b, r in zip(bres[:32], sres))
        log(f"batched SCF of 256 clusters: {t_bscf:.1f} s eager, {t_gscf:.1f} s from graphs "
            f"(max |dE| {dEg:.1e}); 32 single SCFs: {t_sscf32:.1f} s")
    # whole-build model flops (the roofline model of the class kernels) per second
    model = class_flop_model()
    flops = sum(counts[k, 2] * model[k][0] + counts[k, 0] * model[k][1] for k in range(21))
    return {"workload": "256 water clusters, sizes ~U{1..16} (seed 2), molecule i seed 2e6+i, s/p/d basis",
            "molecules": len(mols), "basis_functions": int(nbf.sum()), "quartets_per_build": quartets,
            "load_s": t_load,
            "fp64_ms": t64 * 1e3, "fp64_quartets_per_s": quartets / t64,
            "fp64_model_tflops": flops / t64 / 1e12, "fp64_frac_fp64_peak": flops / t64 / 1e12 / FP64_PEAK_TFLOPS,
            "mixed_model_tflops": flops / tmx / 1e12, "mixed_frac_fp64_peak": flops / tmx / 1e12 / FP64_PEAK_TFLOPS,
            "graph_replay_ms": tg * 1e3, "graph_max_abs_diff": graph_err,
            "mixed_ms": tmx * 1e3, "mixed_quartets_per_s": quartets / tmx, "mixed_max_abs_dF": mixed_err,
            "one_context_per_molecule_ms": tseq * 1e3, "one_context_per_molecule_max_abs_diff": seq_err,
            "speedup_batched_vs_one_by_one": tseq / t64, "speedup_mixed_vs_fp64": t64 / tmx,
            "class_ms_fp64": cms64, "class_ms_mixed": cmsmx,
            "scf": {"batched_s": t_bscf, "batched_converged": int(sum(r["converged"] for r in bres)),
                    "batched_max_iterations": int(max(r["iterations"] for r in bres)),
                    "graph_replay_s": t_gscf, "graph_segments_captured": int(gres[0]["graph_segments"]),
                    "graph_converged": int(sum(r["converged"] for r in gres)),
                    "graph_max_abs_dE_vs_eager": dEg, "speedup_graph_vs_eager": t_bscf / t_gscf,
                    "one_by_one_first32_s": t_sscf32, "one_by_one_256_estimate_s": t_sscf32 * 8,
                    "speedup_batched_vs_one_by_one_est": t_sscf32 * 8 / t_bscf,
                    "max_abs_dE_first32": dE},
            "mixed_quartets_fp32": int(stm.quartets_fp32), "mixed_quartets_fp64": int(stm.quartets_fp64),
            "mixed_fp32_classes": [k for k, v in ptab.items() if v["fp32"]],
            "autotune": autotune.summary(tuning)}


def graphene_bench(args, log):
    """The paper's own workload shape (section 5.2, Table 4): AB-stacked
    graphene bilayers with 15 basis functions per carbon in SP and d shells
    (synthetic exponents), one FP64 Fock build each from a projector density,
    every class in the persistent launch form."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1708_00033_amd import hfx
    out = {"basis": "synthetic split-valence with d: 1s (6 primitives), 2sp (3), 3sp (1), d (1) per carbon",
           "systems": {}}
    sp = torch.cuda.current_stream().cuda_stream
    for name in [x for x in args.graphene.split(",") if x]:
        mol = W.graphene_bilayer(W.GRAPHENE_SIZES[name])
        t0 = time.time()
        ctx = hfx.Context(device=0).load(mol)
        t_load = time.time() - t0
        ctx.set_class_tuning(-1, 32768, 0, 1, -1)
        counts = ctx.class_counts()
        q = int(counts[:, 0].sum())
        D = torch.tensor(W.random_orthonormal_density(mol.nbf, mol.nocc, 7), device="cuda:0")
        F = torch.empty_like(D)
        ctx.build_fock_dev(D.data_ptr(), F.data_ptr(), sp)
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = ctx.build_fock_dev(D.data_ptr(), F.data_ptr(), sp, stats=True)
        dt = time.perf_counter() - t
        if st.quartets_fp64 != q:
            raise RuntimeError(f"graphene {name}: evaluated {st.quartets_fp64} quartets, planned {q}")
        out["systems"][name] = {"atoms": mol.natom, "basis_functions": mol.nbf, "load_s": t_load,
                                "quartets_per_build": q, "integrals_per_build": int(counts[:, 1].sum()),
                                "primitive_quartets_per_build": int(counts[:, 2].sum()), "build_s": dt,
                                "quartets_per_s": q / dt}
        log(f"graphene {name}: {mol.nbf} BF, {q:.3e} quartets, build {dt:.2f} s")
    return out


def large_bench(args, log, fp32_classes=None):
    """512 waters (9728 basis functions), Schwarz tau 1e-11: the full build
    (or one GPU's share, bra pairs r with r mod G = 0, of a G-GPU build) in
    FP64 and mixed (FP32 evaluation on for the classes in fp32_classes, the
    64-water precision autotuner's choice, else for every class; with
    --large-tuned also mixed with FP32 only for the classes where the
    all-FP32 build ran faster), from a
    rank-2560 projector density, every class in the persistent launch form
    with LDS digestion (--large-static: the library's default static form);
    with --large-scf also full SCF."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1708_00033_amd import hfx
    G = args.large_shards
    mol = W.cluster512_config()
    t0 = time.time()
    ctx = hfx.Context(device=0, schwarz_tau=1e-11).load(mol)
    t_load = time.time() - t0
    if not args.large_static:
        ctx.set_class_tuning(-1, 32768, 0, 1, -1)
    counts = ctx.class_counts()
    quartets = int(counts[:, 0].sum())
    log(f"512 waters loaded in {t_load:.1f} s: nbf={ctx.nbf} quartets={quartets:.4e}")
    dev = torch.device("cuda:0")
    D = torch.tensor(W.random_orthonormal_density(mol.nbf, mol.nocc, 33), device=dev)
    G64 = torch.empty_like(D)
    Gmx = torch.empty_like(D)
    sp = torch.cuda.current_stream(dev).cuda_stream
    out = {"workload": f"512-water jittered lattice cluster, seed 3, 5120 shells, 9728 basis functions, "
                       f"Schwarz tau 1e-11, projector density of rank 2560"
                       + ("" if G == 1 else f"; one GPU's share (1/{G} of the bra pairs) of a {G}-GPU build"),
           "nbf": ctx.nbf, "quartets_per_build": quartets, "integrals_per_build": int(counts[:, 1].sum()),
           "primitive_quartets_per_build": int(counts[:, 2].sum()), "load_s": t_load, "shards": G,
           "digest_modes": sorted(set(p["mode"] for p in ctx.plans())),
           "launch_form": "static (library default)" if args.large_static else
                          "persistent, 32768 quartets per task, LDS digestion where the rows fit"}
    Gtn = torch.empty_like(D)
    class_ms = {}
    legs = ((hfx.HFX_PREC_FP64, G64, "fp64"), (hfx.HFX_PREC_MIXED, Gmx, "mixed"))
    if args.large_tuned:
        legs += ((hfx.HFX_PREC_MIXED, Gtn, "mixed_tuned"),)
    for k in range(21):
        ctx.set_class_precision(k, int(fp32_classes is None or hfx.CLASS_NAMES[k] in fp32_classes))
    out["fp32_classes"] = "all" if fp32_classes is None else list(fp32_classes)
    for prec, Go, tag in (() if args.large_no_builds else legs):
        if tag == "mixed_tuned":
            # per class, FP32 only where the mixed build ran the class faster
            for k in range(21):
                ctx.set_class_precision(k, int(class_ms["mixed"][k] < class_ms["fp64"][k]))
        ctx.configure(precision=prec)
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = ctx.build_2e_shard_dev(D.data_ptr(), 2.0, 1.0, 0, G, Go.data_ptr(), sp, stats=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        if args.large_tuned and tag != "mixed_tuned":   # per-class times: one more build with launch events
            ctx.kernel_timing(True)
            ctx.build_2e_shard_dev(D.data_ptr(), 2.0, 1.0, 0, G, Go.data_ptr(), sp)
            torch.cuda.synchronize()
            class_ms[tag], _ = ctx.kernel_times()
            ctx.kernel_timing(False)
        q = int(st.quartets_fp64 + st.quartets_fp32)
        planned_share = int(sum(p["quartets"] for p in ctx.plans())) if G == 1 else None
        if G == 1 and (q != quartets or q != planned_share):
            raise RuntimeError(f"evaluated {q} quartets, planned {quartets}")
        out[tag] = {"share_build_s": dt, "share_quartets": q, "quartets_per_s": q / dt,
                    "quartets_fp32": int(st.quartets_fp32)}
        if tag in class_ms:
            ms = class_ms[tag]
            out[tag]["class_ms"] = {hfx.CLASS_NAMES[k]: round(float(ms[k]), 1) for k in np.argsort(-ms)[:6]}
        log(f"512 waters {tag} share build: {dt:.2f} s, {q:.3e} quartets, {q / dt:.3e} quartets/s")
    if not args.large_no_builds:
        out["mixed"]["max_abs_dG_vs_fp64"] = (Gmx - G64).abs().max().item()
        out["mixed"]["dE_vs_fp64_at_fixed_D"] = float(0.5 * torch.sum(D * (Gmx - G64)).item())
        out["mixed"]["speedup_vs_fp64"] = out["fp64"]["share_build_s"] / out["mixed"]["share_build_s"]
        out["mixed"]["fraction_quartets_fp32"] = out["mixed"]["quartets_fp32"] / max(1, out["mixed"]["share_quartets"])
        if args.large_tuned:
            out["mixed_tuned"]["max_abs_dG_vs_fp64"] = (Gtn - G64).abs().max().item()
            out["mixed_tuned"]["speedup_vs_fp64"] = out["fp64"]["share_build_s"] / out["mixed_tuned"]["share_build_s"]
            out["mixed_tuned"]["fp32_classes"] = [hfx.CLASS_NAMES[k] for k in range(21)
                                                  if class_ms["mixed"][k] < class_ms["fp64"][k]]
        for k in range(21):
            ctx.set_class_precision(k, 1)
    scf_runs = {"none": (), "fp64": ("fp64",), "mixed": ("mixed",), "both": ("fp64", "mixed")}[args.large_scf]
    for tag in scf_runs:
        ctx.configure(precision=hfx.HFX_PREC_FP64 if tag == "fp64" else hfx.HFX_PREC_MIXED, log_level=1)
        r = ctx.scf()   # the library prints one line per iteration (progress of a long run)
        out["scf_" + tag] = {"energy": r["energy"], "iterations": r["iterations"], "converged": r["converged"],
                             "t_total_s": r["t_total_s"], "t_fock_s": r["t_fock_s"]}
        log(f"512 waters SCF {tag}: E={r['energy']:.10f} it={r['iterations']} {r['t_total_s']:.1f} s")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--digest", type=int, default=3,
                    help="digestion: 0 LDS rows of F, 1 global atomics, 2 per-XCD copies, 3 LDS rows of F and D")
    ap.add_argument("--task", type=int, default=8192)
    ap.add_argument("--no-autotune", action="store_true", help="skip the per-class autotuner")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-cluster batched comparison")
    ap.add_argument("--no-large", action="store_true", help="skip the 512-water FP64 and mixed builds")
    ap.add_argument("--large-static", action="store_true",
                    help="512 waters: the library's default static launches instead of the persistent form")
    ap.add_argument("--large-tuned", action="store_true",
                    help="512 waters: also a mixed build with the FP32 kernel only where it ran faster")
    ap.add_argument("--no-graphene", action="store_true", help="skip the graphene bilayers")
    ap.add_argument("--graphene", default="0.5nm,1nm,1.5nm",
                    help="graphene bilayers to build (of 0.5nm, 1nm, 1.5nm, 2nm, 5nm)")
    ap.add_argument("--large-scf", default="none", choices=["none", "fp64", "mixed", "both"],
                    help="with --large: full SCF in these precisions")
    ap.add_argument("--large-no-builds", action="store_true", help="with --large: skip the build timings")
    ap.add_argument("--large-shards", type=int, default=1,
                    help="512 waters: time one GPU's share of a build over this many GPUs (1: the full build)")
    ap.add_argument("--only-large", action="store_true", help="run only the 512-water part")
    ap.add_argument("--tuning", default="", help="profile runs: apply this saved autotuner table")
    ap.add_argument("--save-tuning", default="", help="write the autotuner table here")
    ap.add_argument("--profile", action="store_true",
                    help="profiling run: synthetic projector density, FP64 builds only (class launches on one "
                         "stream), no SCF and no CPU leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 512 MiB device copy (HBM-counter calibration for profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    from paper_1708_00033_amd import hfx

    def log(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    if args.only_large:
        print(json.dumps({"large": large_bench(args, log)}))
        return
    mol = W.cluster64_config()
    ctx = hfx.Context(device=0, digest=args.digest, task_quartets=args.task).load(mol)
    counts = ctx.class_counts()
    log(f"loaded {mol.name}: nbf={ctx.nbf} shells={ctx.nshell} quartets={counts[:, 0].sum():.4e}")
    if args.profile:
        dev = torch.device("cuda:0")
        D = torch.tensor(W.random_orthonormal_density(mol.nbf, mol.nocc, 3), device=dev)
        F = torch.empty_like(D)
        sptr = torch.cuda.current_stream(dev).cuda_stream
        from paper_1708_00033_amd import autotune
        if args.tuning:
            autotune.apply(ctx, autotune.load(args.tuning))
        else:
            ctx.set_class_tuning(-1, *autotune.PREFERRED)
        # launches in order on one stream, as in the builds the per-launch
        # times come from: a dispatch's trace interval and counters are then its own
        ctx.set_streams(1)
        for _ in range(args.warmup + args.steps):
            ctx.build_fock_dev(D.data_ptr(), F.data_ptr(), sptr)
        torch.cuda.synchronize()
        if args.copy_calibration:
            src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device=dev)
            dst = torch.empty_like(src)
            dst.copy_(src)
            torch.cuda.synchronize()
        log(f"profile run done: {args.warmup + args.steps} FP64 builds")
        return
    t0 = time.time()
    r = ctx.scf(e_tol=1e-8, d_rms_tol=1e-7)
    log(f"FP64 SCF: E={r['energy']:.10f} iterations={r['iterations']} converged={r['converged']} "
        f"({time.time() - t0:.1f} s)")
    Dh = r["D"]
    dev = torch.device("cuda:0")
    D = torch.tensor(Dh, device=dev)
    F64 = torch.empty_like(D)
    Fmx = torch.empty_like(D)
    stream = torch.cuda.current_stream(dev)
    sptr = stream.cuda_stream

    tuning = None
    if not args.no_autotune:
        from paper_1708_00033_amd import autotune
        t0 = time.time()
        tuning = autotune.autotune(ctx, D.data_ptr(), F64.data_ptr(), sptr)
        if args.save_tuning:
            autotune.save(tuning, args.save_tuning)
        log(f"autotuned per-class scheduling in {time.time() - t0:.1f} s: "
            f"{autotune.summary(tuning, ['(ss|ss)', '(ps|ss)', '(ds|ss)', '(ps|ps)'])}")

    def timed(nsteps, out, prec):
        ctx.configure(precision=prec)
        for _ in range(args.warmup):
            ctx.build_fock_dev(D.data_ptr(), out.data_ptr(), sptr)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(nsteps):
            ctx.build_fock_dev(D.data_ptr(), out.data_ptr(), sptr)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        # per-launch durations: the same builds again with HIP events around
        # every class launch (the library then keeps the launches in order on
        # this one stream, so each pair of events brackets only its kernel)
        ctx.kernel_timing(True)
        for _ in range(nsteps):
            ctx.build_fock_dev(D.data_ptr(), out.data_ptr(), sptr)
        torch.cuda.synchronize()
        ms, n = ctx.kernel_times()
        plans = ctx.plans()
        ctx.kernel_timing(False)
        st = ctx.build_fock_dev(D.data_ptr(), out.data_ptr(), sptr, stats=True)
        return dt, ms, n, plans, st

    dt64, ms64, n64, plans64, st64 = timed(args.steps, F64, hfx.HFX_PREC_FP64)
    fp32_classes = None
    if not args.no_autotune:   # per class: FP32 kernel on where it is faster
        ctx.configure(precision=hfx.HFX_PREC_MIXED)
        ptab = autotune.autotune_precision(ctx, D.data_ptr(), Fmx.data_ptr(), sptr)
        fp32_classes = [k for k, v in ptab.items() if v["fp32"]]
    dtmx, msmx, nmx, plansmx, stmx = timed(args.steps, Fmx, hfx.HFX_PREC_MIXED)
    quartets = int(counts[:, 0].sum())
    # every planned quartet is evaluated (the timed builds run the same plans as these counted ones)
    for tag, st_ in (("fp64", st64), ("mixed", stmx)):
        if st_.quartets_fp64 + st_.quartets_fp32 != quartets:
            raise RuntimeError(f"{tag} build evaluated {st_.quartets_fp64 + st_.quartets_fp32} quartets, "
                               f"planned {quartets}")
    ctx.configure(precision=hfx.HFX_PREC_FP64)

    # the three digestions of eq. 2 on the same launch form, per class
    digestion = {}
    for dg, name in ((hfx.HFX_DIGEST_LDS_D, "lds_staged_f_and_d_rows"), (hfx.HFX_DIGEST_LDS, "lds_staged"),
                     (hfx.HFX_DIGEST_GLOBAL, "global_atomic"), (hfx.HFX_DIGEST_PRIVATE, "private_per_xcd")):
        ctx.set_class_tuning(-1, 32768, 0, 1, dg)
        ctx.build_fock_dev(D.data_ptr(), F64.data_ptr(), sptr)
        torch.cuda.synchronize()
        ctx.kernel_timing(True)
        t = time.perf_counter()
        for _ in range(2):
            ctx.build_fock_dev(D.data_ptr(), Fmx.data_ptr(), sptr)
        torch.cuda.synchronize()
        dtd = (time.perf_counter() - t) / 2
        msd, nd = ctx.kernel_times()
        ctx.kernel_timing(False)
        digestion[name] = {"build_ms": dtd * 1e3, "class_ms": [round(float(x) / 2, 3) for x in msd],
                           "max_abs_dF_vs_autotuned": (Fmx - F64).abs().max().item()}
    digestion["classes"] = list(hfx.CLASS_NAMES)
    digestion["launch_form"] = "persistent, 32768 quartets per task, no striping (the same for all four)"
    if tuning is not None:
        autotune.apply(ctx, tuning)
    else:
        ctx.set_class_tuning(-1, 0, -1, 0, -1)
    log("digestion comparison: " + ", ".join(f"{k} {v['build_ms']:.1f} ms" for k, v in digestion.items()
                                           if isinstance(v, dict)))

    # several densities in one pass over the integrals (alpha and beta of an unrestricted build)
    Db = torch.tensor(W.random_orthonormal_density(mol.nbf, mol.nocc, 45), device=dev)
    DD = torch.stack([D, Db])
    JJ, KK = torch.empty_like(DD), torch.empty_like(DD)
    ctx.build_jk_multi_dev(2, DD.data_ptr(), JJ.data_ptr(), KK.data_ptr(), sptr)
    torch.cuda.synchronize()
    t = time.perf_counter()
    stm2 = ctx.build_jk_multi_dev(2, DD.data_ptr(), JJ.data_ptr(), KK.data_ptr(), sptr, stats=True)
    t_multi = time.perf_counter() - t
    Jsep, Ksep = torch.empty_like(D), torch.empty_like(D)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for d in range(2):
        ctx.build_2e_dev(DD[d].data_ptr(), 1.0, 0.0, Jsep.data_ptr(), sptr)
        ctx.build_2e_dev(DD[d].data_ptr(), 0.0, -1.0, Ksep.data_ptr(), sptr)
    torch.cuda.synchronize()
    t_sep = time.perf_counter() - t
    multi = {"densities": 2, "one_pass_ms": t_multi * 1e3, "separate_J_and_K_builds_ms": t_sep * 1e3,
             "speedup": t_sep / t_multi, "quartet_evaluations_per_quartet": int(stm2.quartets_fp64) / quartets,
             "max_abs_dK_beta_vs_separate": (KK[1] - Ksep).abs().max().item(),
             "max_abs_dJ_beta_vs_separate": (JJ[1] - Jsep).abs().max().item()}
    log(f"two densities in one pass: {t_multi * 1e3:.1f} ms vs {t_sep * 1e3:.1f} ms for separate J and K builds")
    value = quartets * args.steps / dt64
    value_mx = quartets * args.steps / dtmx
    Fd = (Fmx - F64).abs().max().item()
    dE = float(torch.sum(D * (Fmx - F64)).item())   # E = tr(D (H + F)) at fixed D

    # roofline of the dominant kernel of the FP64 build (the kernel symbol and
    # grid with the most summed time over its launches in a build), measured
    # on its longest launch: one class against one ket list
    model = class_flop_model()
    import gen_eri   # on the path after class_flop_model(); "A": the class's alternative workgroup size

    def launch_shape(p):
        """Kernel symbol and grid of a plan's FP64 launch, as rocprofv3 names them."""
        alt = "A" if p["wgs"] != gen_eri.wg_size(p["cls"]) else ""
        # kernel template digestion: 0 LDS rows (with or without staged D rows), 1 global atomics
        # (into one matrix or the per-XCD copies)
        mode = 0 if p["mode"] in (hfx.HFX_DIGEST_LDS, hfx.HFX_DIGEST_LDS_D) else 1
        if p["persistent"] in (3, 4):
            return f"k_class_kr<Eval{p['cls']}{alt}, {mode}, {p['ket_nprim']}, {p['bras_per_task']}> " \
                   f"grid {p['blocks'] * p['wgs']}"
        form = {0: "k_class", 1: "k_class_persist", 2: "k_class_wave"}[p["persistent"]]
        return f"{form}<Eval{p['cls']}{alt}, {mode}, 0, {p['dstage']}> grid {p['blocks'] * p['wgs']}"

    shape_ms = {}
    for p in plans64:
        shape_ms[launch_shape(p)] = shape_ms.get(launch_shape(p), 0.0) + p["ms"]
    kname = max(shape_ms, key=shape_ms.get)
    # launches of one class against several ket lists can share a kernel and grid: the
    # profiles key each by its position among them in a build
    same = [q for q in plans64 if launch_shape(q) == kname]
    dom = max(same, key=lambda p: p["ms"])
    per_prim, per_q, nint = model[dom["cls"]]
    flops_launch = dom["prim"] * per_prim + dom["quartets"] * per_q
    avg_ms = dom["ms"] / max(dom["launches"], 1)
    achieved = flops_launch / (avg_ms * 1e-3) / 1e12
    kname_launch = f"{kname} launch {next(i for i, q in enumerate(same) if q is dom) + 1} of {len(same)}"
    total_flops = sum(counts[k, 2] * model[k][0] + counts[k, 0] * model[k][1] for k in range(21))
    traffic = None
    counted = None
    prof = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if os.path.exists(prof):
        with open(prof) as fh:
            pj = json.load(fh)
        # per profiled launch: {kernel: {"hbm_bytes_per_launch": ..., "counted_fp64_flops_per_launch": ...}}
        kernels = pj.get("kernels", {pj.get("kernel"): pj})
        if pj.get("source_hash") == source_hash() and kname_launch in kernels:
            traffic = kernels[kname_launch].get("hbm_bytes_per_launch")
            cf = kernels[kname_launch].get("counted_fp64_flops_per_launch")
            if cf:
                # FP64 VALU instructions counted by the hardware (ADD, MUL,
                # transcendental: 64 flops per wave instruction, FMA: 128),
                # over the live HIP-event duration of the launch
                ach = cf / (avg_ms * 1e-3) / 1e12
                counted = {"flops_per_launch": cf, "achieved": ach, "frac": ach / FP64_PEAK_TFLOPS,
                           "note": "every lane of a counted wave instruction taken as active"}
    res = {
        "metric": "screened ERI quartets/s + Fock-build time, FP64 vs mixed @1e-6 Eh, 1 GPU",
        "value": value,
        "unit": "quartets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt64 / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded water cluster, synthetic even-tempered basis)",
        "config": {"workload": "64-water jittered lattice cluster, seed 1, 640 shells, 1216 Cartesian basis "
                               "functions, Schwarz tau 1e-10, converged FP64 SCF density",
                   "nbf": ctx.nbf, "shells": ctx.nshell, "quartets_per_build": quartets,
                   "integrals_per_build": int(counts[:, 1].sum()),
                   "primitive_quartets_per_build": int(counts[:, 2].sum()),
                   "digest": {0: "lds-staged F rows", 1: "global-atomic", 2: "private per-XCD copies",
                              3: "lds-staged F and D rows"}[args.digest], "task_quartets": args.task},
        "mixed": {"value": value_mx, "unit": "quartets/s", "ms_per_step": dtmx / args.steps * 1e3,
                  "speedup_vs_fp64": dt64 / dtmx, "fp32_tau": 1e-7, "quartets_fp32": int(stmx.quartets_fp32),
                  "quartets_fp64": int(stmx.quartets_fp64), "max_abs_dF_vs_fp64": Fd,
                  "fp32_classes": fp32_classes,
                  "dE_vs_fp64_at_fixed_D": dE,
                  "build_flops_model_tflops": total_flops / (dtmx / args.steps) / 1e12,
                  "build_frac_fp64_peak": total_flops / (dtmx / args.steps) / 1e12 / FP64_PEAK_TFLOPS},
        "roofline": {"bound": "alu", "kernel": kname, "launch": kname_launch, "class": hfx.CLASS_NAMES[dom["cls"]],
                     "kernel_ms_per_build": shape_ms[kname] / max(dom["launches"], 1),
                     "ket_nprim": dom["ket_nprim"], "achieved": achieved,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": traffic, "counted": counted,
                     "avg_launch_ms": avg_ms, "flops_per_launch": float(flops_launch),
                     "quartets_per_launch": dom["quartets"], "primitive_quartets_per_launch": dom["prim"]},
        "build_flops_model_tflops": total_flops / (dt64 / args.steps) / 1e12,
        "build_frac_fp64_peak": total_flops / (dt64 / args.steps) / 1e12 / FP64_PEAK_TFLOPS,
        "class_ms_fp64": {hfx.CLASS_NAMES[k]: round(ms64[k] / max(n64[k], 1), 3) for k in np.argsort(-ms64)[:8]},
        "class_ms_mixed": {hfx.CLASS_NAMES[k]: round(msmx[k] / max(nmx[k], 1), 3) for k in np.argsort(-msmx)[:8]},
        "scf": {"energy": r["energy"], "iterations": r["iterations"]},
        "autotune": None if tuning is None else autotune.summary(tuning),
        "digestion": digestion,
        "multi_density": multi,
    }
    if not args.no_batch:
        log("batched builds: 256 clusters of 1-16 waters ...")
        res["batched"] = batched_bench(args, log)
    if not args.no_graphene:
        res["graphene"] = graphene_bench(args, log)
    if not args.no_large:
        res["large"] = large_bench(args, log, fp32_classes)
    if args.copy_calibration:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        res["copy_calibration_bytes"] = src.numel() * 8
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        cb = cpu_baseline(mol, Dh)
        res["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample", "host", "one_thread")}
    print(json.dumps(res))


if __name__ == "__main__":
    main()
