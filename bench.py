"""Benchmark of the Sternheimer chi0 / Lanczos dielectric hot path on one MI355X.

One step = the whole hot path on the silane-sized molecule-in-a-box workload
(L = 20 bohr, 48^3 grid, ecut 10 Ha, 12,053 plane waves, 5 Gaussian wells,
4 valence bands): a 64-step Lanczos basis of eps(0) - 1 built with full
reorthogonalisation (64 static chi0 applies), then eps(z) - 1 projected on that
basis at 32 frequencies (16 imaginary, 0..2 Ha; 16 real, 0..1 Ha with
0.1 eV broadening): 32 * 64 = 2,048 distinct chi0 applies (the recursion's 64
static applies are the z = 0 column of the projection).  `value` is chi0
applies per second of the mixed-precision path (FP32 transforms and projector
inside FP64 refinement) with the projection's 32 frequencies solved from one
Lanczos recursion per column and band (multi-shift, FP64), and the kinetic
preconditioner with the shifted-pair imaginary axis for the single-frequency
solves of the Lanczos basis; the FP64 path and both precisions in the
unpreconditioned form (squared-equation CG on the imaginary axis, plain SQMR
on the real axis) are timed beside it.  The projection of finished Lanczos
vectors runs on a second stream while the recursion continues
(lgw_lanczos_project); the two phases one after the other are timed once
after warm-up for the breakdown.  Inputs are synthetic and resident in HBM
before the timed region starts.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "chi0*v applies/sec & Sternheimer H*psi GB/s, mixed vs FP64 at 1e-6 rel err"
HBM_PEAK_GBPS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def hpsi_model_bytes(npw: int, ncols: int, N: int, elem: int) -> float:
    """Algorithmic bytes of one pruned H application (three passes):
    sphere read, column write+read, column read+write, sphere write plus the
    second read of the input for the kinetic term; the potential plane is
    shared by all systems and comes from cache."""
    return elem * (3.0 * npw + 4.0 * ncols * N)


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ["k_fft.hip", "fft_lds.h", "common.h", "k_solve.hip"]:
        with open(os.path.join(ROOT, "paper_1408_3036_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, mode: str, model_bytes_per_launch: float):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary
    (FETCH_SIZE and WRITE_SIZE per system of the batched launches, each
    scaled by the factor that makes a plain 1 GiB copy read as 1 GiB), scaled
    to the systems of this run's launches; None if the transform sources
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_silane48.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    ent = rec.get("kernels", {}).get(kernel)
    if not ent or rec.get("source_hash") != kernel_source_hash():
        return None
    systems = (model_bytes_per_launch - ent["model_bytes_fixed"]) / ent["model_bytes_per_system"]
    return round(ent["hbm_bytes_per_system"] * systems + ent["model_bytes_fixed"])


def _oracle_sample(task):
    """One worker of the CPU baseline: the oracle's matrix-free Sternheimer
    chi0 (O2) of one column at the sample's frequencies, single-threaded."""
    L, N, ecut, V, psi, eps, zs, x = task
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=1)
    except ImportError:
        pass
    sys.path.insert(0, ROOT)
    from oracle.pw import Basis
    from oracle.sternheimer import MatrixFree
    mf = MatrixFree(Basis(L, N, ecut), V, psi, eps)
    t = time.perf_counter()
    out = [mf.chi0(complex(z), x) for z in zs]
    return np.array(out), time.perf_counter() - t


def cpu_cores() -> int:
    """Host cores this process may run on, capped at the 16-core share of one
    GPU on the benchmark hosts."""
    return max(1, min(len(os.sched_getaffinity(0)), 16))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, zs_sample, xs, cores):
    """The oracle's matrix-free Sternheimer chi0 (O2) on the columns xs at the
    frequencies zs_sample, one column per task over `cores` worker processes
    (each single-threaded: numpy's FFT is, and BLAS is pinned to one thread).
    Returns (results [n_cols, n_z, N^3], wall seconds, summed worker seconds)."""
    import multiprocessing as mp
    tasks = [(w.L, w.N, w.ecut, w.V, w.psi, w.eps, list(zs_sample), x) for x in xs]
    ctx = mp.get_context("spawn")
    with ctx.Pool(processes=min(cores, len(tasks))) as pool:
        pool.map(_oracle_sample, tasks[:1])            # worker start-up and imports, untimed
        t = time.perf_counter()
        res = pool.map(_oracle_sample, tasks)
        wall = time.perf_counter() - t
    return np.array([r[0] for r in res]), wall, sum(r[1] for r in res)


def rocpd_counters(db: str, pattern: str):
    """Per dispatch of the kernels whose name contains `pattern` in a
    rocprofv3 results database: {dispatch_id: (systems, {counter: value},
    duration_ns)}; systems is the grid's y extent (the system count of the
    batched launches)."""
    import sqlite3
    con = sqlite3.connect(db)
    out = {}
    for disp, name, gy, cname, val, dur in con.execute(
            "select dispatch_id, kernel_name, grid_size_y, counter_name, value, duration "
            "from counters_collection"):
        if pattern not in name:
            continue
        ent = out.setdefault(disp, [int(gy), {}, dur])
        ent[1][cname] = ent[1].get(cname, 0.0) + float(val)
    return out


def summarise_traffic(fetch_db, write_db, calib_fetch_db, calib_write_db, kernel, model_per_system,
                      model_fixed, min_systems=16):
    """HBM bytes per system of `kernel` from FETCH_SIZE and WRITE_SIZE runs
    (KiB per dispatch), each scaled by the factor that makes the same counter
    read 1 GiB for a plain 1 GiB device copy (bench.py --calib-copy); only
    dispatches of at least min_systems systems are averaged.  The bytes read
    once per launch (model_fixed: the potential plane) are taken off each
    dispatch's scaled fetch before the division, so the per-system figures
    compare with model_per_system alone."""
    def totals(db, cname):
        rows = [(g, c[cname]) for g, c, _ in rocpd_counters(db, kernel).values() if cname in c and g >= min_systems]
        return sum(v for _, v in rows) * 1024.0, sum(g for g, _ in rows), len(rows)

    def calib(db, cname):
        rows = [c[cname] for g, c, _ in rocpd_counters(db, "copyBuffer").values() if cname in c]
        rows = rows or [c[cname] for g, c, _ in rocpd_counters(db, "").values() if cname in c]
        return (1 << 30) / (max(rows) * 1024.0)
    cf, cw = calib(calib_fetch_db, "FETCH_SIZE"), calib(calib_write_db, "WRITE_SIZE")
    F, sf, nf = totals(fetch_db, "FETCH_SIZE")
    W, sw, nw = totals(write_db, "WRITE_SIZE")
    f = (F * cf - nf * model_fixed) / sf
    w = W * cw / sw
    return {"kernel": kernel, "dispatches": [nf, nw], "systems": [sf, sw],
            "fetch_bytes_per_system": round(f), "write_bytes_per_system": round(w),
            "hbm_bytes_per_system": round(f + w),
            "calibration": {"fetch_scale": cf, "write_scale": cw},
            "model_bytes_per_system": model_per_system, "model_bytes_fixed": model_fixed,
            "counters_over_model": round((f + w) / model_per_system, 3)}


def bench_large72(log_fn):
    """The large-molecule workload at its shape: block Lanczos, 8-vector blocks
    to 256 vectors, then eps(z) - 1 on that basis at the 32 imaginary
    frequencies (mixed precision with the fast solver options, multi-shift
    projection).  Returns the record for the JSON line."""
    import torch
    from paper_1408_3036_amd import Lgw
    from synthetic import make_workload, random_potentials
    w = make_workload(3)
    seeds = torch.from_numpy(random_potentials(w.N, 8, (14083036, 3, 0, 80)))
    zs = list(w.z)
    lg = Lgw(w.L, w.N, w.ecut, torch.from_numpy(w.V), torch.from_numpy(w.psi), w.eps, precision="mixed",
             tol=1e-10, precond=True, imag_form="shifted", multishift=True)
    try:
        lg.block_lanczos(seeds, 2, want_Q=False)          # warm-up (workspace, graphs)
        torch.cuda.synchronize()
        t = time.perf_counter()
        A, B, Q, nd = lg.block_lanczos(seeds, 32)
        torch.cuda.synchronize()
        t_l = time.perf_counter() - t
        t = time.perf_counter()
        E = lg.project(Q, zs)
        torch.cuda.synchronize()
        t_p = time.perf_counter() - t
        npw = lg.npw
    finally:
        lg.close()
    n_apply = 256 + (len(zs) - 1) * 256      # the z = 0 block of E is the recursion's (distinct applies)
    log_fn(f"[large-72] block Lanczos {t_l:.2f}s, projection {t_p:.2f}s")
    return {"workload": f"{w.name}: L={w.L} bohr, {w.N}^3 grid, ecut {w.ecut} Ha, {npw} PW, {w.n_wells} wells, "
                        f"n_v={w.n_v}; block Lanczos 32 x 8 vectors + eps(z)-1 at {len(zs)} imaginary z",
            "chi0_applies": n_apply, "seconds": round(t_l + t_p, 3),
            "chi0_applies_per_s": round(n_apply / (t_l + t_p), 1),
            "block_lanczos_s": round(t_l, 3), "projection_s": round(t_p, 3),
            "band_systems": 16 * n_apply,
            "how": "mixed precision (FP32 transforms inside FP64 refinement) with the kinetic preconditioner "
                   "for the 256 static columns, multi-shift FP64 recursions for the projection; the projection "
                   "recomputes z = 0, counted once"}


def bench_uneven(log_fn, n_box: int = 32):
    """The batched uneven-systems workload: every box runs a 32-step Lanczos
    and eps(z) - 1 at its 8 imaginary frequencies (lanczos_project), first one
    box after the other (per-system rates), then all boxes at once, one host
    thread and stream per box (aggregate rate).  Ground states are built over
    the host cores beforehand."""
    import tempfile
    import shutil
    import threading
    import torch
    from paper_1408_3036_amd import Lgw
    from synthetic import random_potentials
    from synthetic.boxes import make_uneven_boxes
    d = tempfile.mkdtemp(prefix="lgw_uneven_")
    try:
        t = time.perf_counter()
        boxes = make_uneven_boxes(d, n_box)
        log_fn(f"[uneven] {n_box} boxes built in {time.perf_counter() - t:.1f}s")
        lgs, q0s = [], []
        for bx in boxes:
            V = torch.from_numpy(np.load(bx["pre"] + "_V.npy"))
            psi = torch.from_numpy(np.load(bx["pre"] + "_psi.npy"))
            eps = np.load(bx["pre"] + "_eps.npy")
            # 32 contexts (and their two projection twins each) share the GPU's
            # memory: a 1 GB workspace cap each bounds the multi-shift chunks
            lgs.append(Lgw(bx["L"], bx["N"], bx["ecut"], V, psi, eps, precision="mixed", tol=1e-10,
                           precond=True, imag_form="shifted", multishift=True, mem_budget_gb=1.0))
            q0s.append(torch.from_numpy(random_potentials(bx["N"], 1, (14083036, 4, bx["sys"], 99))[0]).cuda())
        zs = list(boxes[0]["z"])
        k = 32
        n_apply = k + (len(zs) - 1) * k
        try:
            for lg, q0 in zip(lgs, q0s):                     # warm-up
                lg.lanczos_project(q0, k, zs, want_Q=False)
            torch.cuda.synchronize()
            per = []
            for lg, q0 in zip(lgs, q0s):
                t = time.perf_counter()
                lg.lanczos_project(q0, k, zs, want_Q=False)
                torch.cuda.synchronize()
                per.append(time.perf_counter() - t)
            errs = []

            def run(i):
                try:
                    lgs[i].lanczos_project(q0s[i], k, zs, want_Q=False)
                except Exception as e:          # reported, not raised in the thread
                    errs.append(repr(e))
            torch.cuda.synchronize()
            t = time.perf_counter()
            th = [threading.Thread(target=run, args=(i,)) for i in range(len(lgs))]
            for x in th:
                x.start()
            for x in th:
                x.join()
            torch.cuda.synchronize()
            conc = time.perf_counter() - t
        finally:
            for lg in lgs:
                lg.close()
    finally:
        shutil.rmtree(d, ignore_errors=True)
    seq = sum(per)
    log_fn(f"[uneven] one after the other {seq:.2f}s, all at once {conc:.2f}s")
    return {"workload": f"{n_box} boxes, grids {sorted(set(b['N'] for b in boxes))}, n_v "
                        f"{min(b['n_v'] for b in boxes)}..{max(b['n_v'] for b in boxes)}; per box {k}-step "
                        f"Lanczos + eps(z)-1 at {len(zs)} imaginary z",
            "chi0_applies": n_apply * n_box,
            "aggregate_chi0_applies_per_s": round(n_apply * n_box / conc, 1),
            "sequential_chi0_applies_per_s": round(n_apply * n_box / seq, 1),
            "concurrent_over_sequential": round(seq / conc, 3),
            "errors": errs,
            "per_system": [{"sys": b["sys"], "N": b["N"], "n_v": b["n_v"], "seconds": round(p, 4),
                            "chi0_applies_per_s": round(n_apply / p, 1)} for b, p in zip(boxes, per)],
            "how": "mixed precision, fast solver options, multi-shift projection; per-system rates from the "
                   "boxes run one after the other, the aggregate from all boxes at once (one host thread, "
                   "context and stream per box)"}


def bench_sigma(w, lg_kw, q0, log_fn):
    """Correlation self-energy of the highest valence state on the silane-sized
    basis: sigma_N, sigma_N0 at 8 Gauss-Legendre frequencies of the half line,
    the Lorentzian term (a = 1 Ha) and the residues (4 Lanczos steps per pole)."""
    import torch
    from paper_1408_3036_amd import Lgw
    t_nodes, t_w = np.polynomial.legendre.leggauss(8)
    ws = (1 + t_nodes) / (1 - t_nodes)
    wts = t_w * 2 / (1 - t_nodes) ** 2
    lg = Lgw(w.L, w.N, w.ecut, torch.from_numpy(w.V), torch.from_numpy(w.psi), w.eps, **lg_kw)
    try:
        _, _, Q, kd = lg.lanczos(q0, 64)
        e, delta = w.n_v - 1, -0.1
        lg.sigma_traces(e, delta, Q[:8], ws[:2])     # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        sN, sN0, sA = lg.sigma_traces(e, delta, Q, ws)
        t_tr = time.perf_counter() - t
        t = time.perf_counter()
        sP, npl = lg.sigma_residues(e, delta, 4)
        t_res = time.perf_counter() - t
    finally:
        lg.close()
    sc = float(np.sum(wts * (sN - sN0)) / np.pi + sA + sP)
    log_fn(f"[sigma] traces {t_tr:.2f}s, residues {t_res:.2f}s, Sigma_c {sc:.6f} Ha")
    return {"state": "highest valence", "delta_Ha": delta, "basis": kd, "frequencies": len(ws),
            "traces_s": round(t_tr, 3), "residues_s": round(t_res, 3), "poles": npl,
            "sigma_c_Ha": sc, "sigma_A_Ha": sA, "sigma_P_Ha": sP,
            "how": "lgw_sigma_traces (E(z) at 9 frequencies, shift-Lanczos of H for the 8 integrand "
                   "frequencies, one static solve per basis vector for the Lorentzian term) and "
                   "lgw_sigma_residues on the 64-vector static Lanczos basis"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--lanczos", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", choices=["both", "fp64", "mixed"], default="both")
    ap.add_argument("--solver", choices=["both", "fast", "paper"], default="both",
                    help="fast: kinetic preconditioner + shifted pair on the imaginary axis; "
                         "paper: unpreconditioned, squared form on the imaginary axis")
    ap.add_argument("--multishift", type=int, default=1,
                    help="1 (default): the fast form also solves all frequencies of a call from one "
                         "Lanczos recursion per (column, band); 0: one Krylov solve per shift")
    ap.add_argument("--no-breakdown", action="store_true",
                    help="skip the sequential Lanczos / projection pass (profiling runs: every "
                         "launch then has the timed step's shape)")
    ap.add_argument("--no-model", action="store_true",
                    help="skip the model-operator step measured beside the headline")
    ap.add_argument("--no-recycle", action="store_true",
                    help="skip the frequency-recycling measurement beside the headline mode")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run only a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--summarise-traffic", nargs=4, metavar=("FETCH_DB", "WRITE_DB", "COPY_FETCH_DB", "COPY_WRITE_DB"),
                    help="print the plane pass's HBM traffic summary from rocprofv3 --pmc databases")
    ap.add_argument("--counter-summary", nargs="+", metavar="DB_THEN_PATTERNS",
                    help="print per-kernel means of a rocprofv3 --pmc database (kernel-name substrings follow)")
    ap.add_argument("--mixed-tol", type=float, default=1e-8,
                    help="relative residual tolerance of every solve in the mixed-precision path "
                         "(1e-8 keeps the mixed results at least ten times inside the 1e-6 target "
                         "of the metric: alpha, beta and E(z) against the FP64 path are reported)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the large-72, uneven-batch and self-energy measurements beside the headline")
    args = ap.parse_args()
    if args.summarise_traffic:
        # profiles/traffic_silane48.json from four rocprofv3 databases:
        # FETCH_SIZE and WRITE_SIZE of the bench, then of the 1 GiB copy
        from synthetic import make_workload
        fdb, wdb, cfdb, cwdb = args.summarise_traffic
        w = make_workload(2, with_ground_state=False)
        N = w.N
        m = np.arange(-N // 2 + 1, N // 2)
        kxy = 0.5 * (2 * np.pi / w.L) ** 2 * (m[:, None] ** 2 + m[None, :] ** 2)
        ncols = int(np.count_nonzero(kxy <= w.ecut))      # z-columns holding plane waves
        rec = {"source_hash": kernel_source_hash(), "workload": "silane-48",
               "kernels": {"plane_hv_f64": summarise_traffic(fdb, wdb, cfdb, cwdb, "k_plane_hv<double",
                                                             16.0 * 2 * N * ncols, 8.0 * N ** 3)},
               "model": "plane pass per system: e 2 N ncols (the columns read and written once); "
                        "the potential plane (8 N^3 per launch) once per launch"}
        print(json.dumps(rec, indent=1))
        return
    if args.counter_summary:
        # per-kernel means of every counter in a rocprofv3 --pmc database
        db = args.counter_summary[0]
        pats = args.counter_summary[1:] or [""]
        import collections
        for pat in pats:
            rows = rocpd_counters(db, pat)
            import sqlite3
            names = {}
            con = sqlite3.connect(db)
            for disp, name in con.execute("select dispatch_id, kernel_name from counters_collection"):
                names[disp] = name
            by = collections.defaultdict(list)
            for disp, (gy, cs, dur) in rows.items():
                import re
                mk = re.search(r"(k_\w+(<[^()]*>)?)", names[disp])
                by[mk.group(1) if mk else names[disp][:60]].append((gy, cs, dur))
            for kname, lst in sorted(by.items(), key=lambda t: -sum(x[2] for x in t[1])):
                cn = sorted(set(c for _, cs, _ in lst for c in cs))
                line = {c: sum(cs.get(c, 0.0) for _, cs, _ in lst) / len(lst) for c in cn}
                print(f"{kname}: dispatches {len(lst)}, mean systems {sum(g for g, _, _ in lst) / len(lst):.1f}, "
                      f"mean duration {sum(d for _, _, d in lst) / len(lst) / 1e3:.2f} us")
                for c in cn:
                    print(f"    {c:32s} {line[c]:.6g} per dispatch")
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calib_copy:
        a = torch.ones(1 << 26, dtype=torch.complex128, device="cuda")   # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": a.numel() * 16, "launches": 3}))
        return

    from paper_1408_3036_amd import Lgw
    from synthetic import make_workload, random_potentials

    t0 = time.time()
    w = make_workload(2)
    log(f"workload {w.name}: N={w.N} L={w.L} ecut={w.ecut} n_v={w.n_v} gap={w.gap:.3f} "
        f"({time.time() - t0:.1f}s)")
    zs = w.z
    k = args.lanczos
    q0 = torch.from_numpy(random_potentials(w.N, 1, (14083036, 2, 0, 99))[0]).cuda()
    V = torch.from_numpy(w.V).cuda()
    psi = torch.from_numpy(w.psi).cuda()
    # sampled oracle check: one real-valued potential at four frequencies
    x_s = random_potentials(w.N, 1, (14083036, 2, 0, 7))[0]
    z_s = np.array([0.0, 0.13j, 2.0j, 0.5 + 1j * zs[-1].imag])

    results = {}
    precs = ["fp64", "mixed"] if args.only == "both" else [args.only]
    forms = ["fast", "paper"] if args.solver == "both" else [args.solver]
    runs = [(p if f == "fast" else f"{p}_paper", p, f) for f in forms for p in precs]
    for mode, prec, form in runs:
        kw = dict(tol=1e-13) if prec == "fp64" else dict(precision="mixed", tol=args.mixed_tol)
        if form == "fast":
            kw.update(precond=True, imag_form="shifted")
            if args.multishift:
                kw.update(multishift=True)
        lg = Lgw(w.L, w.N, w.ecut, V, psi, w.eps, **kw)
        tl = tp = 0.0
        for i in range(args.warmup):
            t = time.time()
            lg.lanczos_project(q0, k, zs, want_Q=False)
            torch.cuda.synchronize()
            log(f"[{mode}] warmup {i}: {time.time() - t:.2f}s")
        kt_iso = None
        if args.warmup and not args.no_breakdown:
            # the two phases one after the other, timed for the breakdown only;
            # kernel timings here see each kernel alone on the GPU
            lg.profile(True)
            s0 = time.perf_counter()
            a, b, Q, kd = lg.lanczos(q0, k)
            torch.cuda.synchronize()
            s1 = time.perf_counter()
            lg.project(Q, zs)
            torch.cuda.synchronize()
            tl, tp = s1 - s0, time.perf_counter() - s1
            kt_iso = lg.kernel_timing()
        lg.profile(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        it = ha = 0
        for i in range(args.steps):
            s0 = time.perf_counter()
            a, b, Q, E, kd = lg.lanczos_project(q0, k, zs)
            torch.cuda.synchronize()
            st_ = lg.stats()
            it += st_["total_iters"]
            ha += st_["total_happly"]
            log(f"[{mode}] step {i}: {time.perf_counter() - s0:.4f}s iters {st_['total_iters']} "
                f"H {st_['total_happly']}")
        el = time.perf_counter() - t
        kt = lg.kernel_timing()
        lg.profile(False)
        rec = None
        if form == "fast" and not args.no_recycle and (prec == "mixed" or args.only == "fp64"):
            # frequency recycling at the imaginary frequencies, on the same static basis
            idx = [i for i, z in enumerate(zs) if z.real == 0.0]
            wi = [zs[i].imag for i in idx]
            lg.lanczos_recycle(q0, k, wi, want_Q=False)
            torch.cuda.synchronize()
            t_r = time.perf_counter()
            _, _, _, Er, kr = lg.lanczos_recycle(q0, k, wi, want_Q=False)
            torch.cuda.synchronize()
            t_r = time.perf_counter() - t_r
            Er, Ed = Er.cpu().numpy(), E.cpu().numpy()[idx]
            dev = [float(np.linalg.norm(Er[j] - Ed[j]) / np.linalg.norm(Ed[j])) for j in range(len(idx))]
            rec = dict(seconds=t_r, dev=dev, n_w=len(idx), k=kr)
            log(f"[{mode}] recycling: {t_r:.3f}s for {len(idx)} imaginary frequencies, "
                f"max rel. deviation {max(dev):.2e}")
        dn_s = lg.chi0_apply(torch.from_numpy(x_s[None]), z_s).cpu().numpy()[:, 0]
        plain = None
        if mode == "fp64" or (mode == "fp64_paper" and "fp64" not in [r[0] for r in runs]):
            # the plain path: one chi0 apply (one column, one frequency) per call
            xs = torch.from_numpy(random_potentials(w.N, 2, (14083036, 2, 0, 8))).cuda()
            zp = [z_s[0], z_s[1], z_s[2], z_s[3]]
            lg.chi0_apply(xs[:1], zp[:1])
            torch.cuda.synchronize()
            tp0 = time.perf_counter()
            for j in range(2):
                for zz in zp:
                    lg.chi0_apply(xs[j:j + 1], [zz])
            torch.cuda.synchronize()
            plain = 8 / (time.perf_counter() - tp0)
        # accuracy: eps(z)-1 projected on the FP64 path's Lanczos basis
        E_ref_basis = None
        if prec == "mixed" and "fp64" in results:
            E_ref_basis = lg.project(results["fp64"]["Q"], zs).cpu().numpy()
        results[mode] = dict(Q=Q, E_fp64_basis=E_ref_basis, plain=plain, elapsed=el, lanczos_s=tl, project_s=tp,
                             kt_iso=kt_iso,
                             alpha=a.cpu().numpy(),
                             beta=b.cpu().numpy(), E=E.cpu().numpy(), iters=it, happly=ha,
                             npw=lg.npw, ncols=lg.ncols, kt=kt, dn_s=dn_s, k_done=kd, rec=rec)
        lg.close()

    model = None
    if not args.no_model:
        # the model dielectric operator of Sec. V (H -> T) on the same step
        lg = Lgw(w.L, w.N, w.ecut, V, psi, w.eps, model=True)
        lg.lanczos_project(q0, k, zs, want_Q=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        lg.lanczos_project(q0, k, zs, want_Q=False)
        torch.cuda.synchronize()
        model = time.perf_counter() - t
        lg.close()
        log(f"[model] step: {model:.3f}s")
    # distinct chi0 applies per step: the k static applies of the recursion
    # serve as the z = 0 column of E(z), so the other len(zs) - 1 frequencies
    # add k applies each (z = 0 is one of the 32 frequencies)
    n_apply = k + (len(zs) - 1) * k if any(z == 0 for z in zs) else k + len(zs) * k
    extras = {}
    if not args.no_extra:
        for name, fn in (("large72", lambda: bench_large72(log)), ("uneven32", lambda: bench_uneven(log)),
                         ("sigma", lambda: bench_sigma(w, dict(tol=1e-13, precond=True, imag_form="shifted",
                                                                multishift=True), q0, log))):
            try:
                extras[name] = fn()
            except Exception as e:      # a failed extra is reported; it does not cost the headline line
                extras[name] = {"error": repr(e)}
                log(f"[{name}] failed: {e!r}")
    main_mode = [m for m in ("mixed", "fp64", "mixed_paper", "fp64_paper") if m in results][0]
    main_prec = "mixed" if main_mode.startswith("mixed") else "fp64"
    r = results[main_mode]
    ms = 1e3 * r["elapsed"] / args.steps
    value = n_apply * args.steps / r["elapsed"]
    out = {"metric": METRIC, "value": round(value, 2), "unit": "chi0-applies/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 1),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": (("f64 projection, f32+f64-refine basis" if args.multishift and not main_mode.endswith("_paper")
                      else "f32+f64-refine") if main_prec == "mixed" else "f64"), "data": "synthetic",
           "config": {"workload": f"{w.name}: L={w.L} bohr, {w.N}^3 grid, ecut {w.ecut} Ha, "
                                  f"{r['npw']} PW, {w.n_wells} Gaussian wells, n_v={w.n_v}; "
                                  f"{k}-step Lanczos + eps(z)-1 at {len(zs)} z "
                                  f"(16 imaginary 0..2 Ha, 16 real 0..1 Ha + 0.1 eV)",
                      "chi0_applies_per_step": n_apply,
                      "solver": (("multi-shift Lanczos for the 32 frequencies (one recursion per "
                                  "column and band, FP64, every shift checked by its true residual); "
                                  if args.multishift else "") +
                                 "kinetic preconditioner (symmetric diagonal scaling), imaginary axis "
                                 "as two shifted SQMR systems" if not main_mode.endswith("_paper")
                                 else "unpreconditioned; squared-form CG on the imaginary axis")}}
    # roofline of the dominant kernel of the main path (HIP events, live)
    kt = r["kt"]
    dom = max(kt, key=lambda n: kt[n]["total_ms"])
    d = kt[dom]
    ach = d["model_bytes"] / (d["total_ms"] * 1e-3) / 1e9
    trf = measured_traffic(dom, main_prec, d["model_bytes"] / max(d["launches"], 1))
    out["roofline"] = {"bound": "hbm", "kernel": f"k_{dom}", "achieved": round(ach, 1),
                       "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBPS, 4),
                       "traffic": trf, "launches": d["launches"],
                       "avg_launch_us": round(1e3 * d["total_ms"] / max(d["launches"], 1), 2),
                       "model_bytes_per_launch": round(d["model_bytes"] / max(d["launches"], 1)),
                       "streams": "recursion + 2 projection streams share the GPU; launch durations "
                                  "include that sharing"}
    iso = (r.get("kt_iso") or {}).get(dom)
    if iso and iso["total_ms"] > 0:
        a_iso = iso["model_bytes"] / (iso["total_ms"] * 1e-3) / 1e9
        out["roofline"]["isolated"] = {
            "achieved": round(a_iso, 1), "frac": round(a_iso / HBM_PEAK_GBPS, 4),
            "launches": iso["launches"],
            "avg_launch_us": round(1e3 * iso["total_ms"] / max(iso["launches"], 1), 2),
            "how": "same kernel, HIP events, in the one-after-the-other Lanczos and projection pass "
                   "(one stream, 64 columns per projection batch)"}
    for mode, rr in results.items():
        kt = rr["kt"]
        suf = "f64" if mode.startswith("fp64") else "f32"
        # every timed transform launch of the step, whatever its precision
        # (the headline's multi-shift projection runs its transforms in FP64
        # under the mixed option); each carries its own model bytes
        hk = [f"{n}_{p}" for p in ("f64", "f32") for n in ("zinv", "plane_hv", "zfwd") if f"{n}_{p}" in kt]
        h_ms = sum(kt[n]["total_ms"] for n in hk)
        h_gbps = sum(kt[n]["model_bytes"] for n in hk) / (h_ms * 1e-3) / 1e9 if h_ms else None
        dst = out.setdefault("paper_form", {}) if mode.endswith("_paper") else out
        dst[mode.replace("_paper", "")] = {"chi0_applies_per_s": round(n_apply * args.steps / rr["elapsed"], 2),
                     "step_s": round(rr["elapsed"] / args.steps, 3),
                     "sequential_lanczos_s": round(rr["lanczos_s"], 3),
                     "sequential_project_s": round(rr["project_s"], 3),
                     "krylov_iters": int(rr["iters"] / args.steps),
                     "h_applies": int(rr["happly"] / args.steps),
                     "hpsi_GBps": round(h_gbps, 1) if h_gbps else None,
                     "hpsi_kernels": hk,
                     "hpsi_frac_hbm": round(h_gbps / HBM_PEAK_GBPS, 4) if h_gbps else None,
                     "hpsi_model_bytes": hpsi_model_bytes(rr["npw"], rr["ncols"], w.N, 16 if suf == "f64" else 8),
                     "kernel_ms": {n: round(v["total_ms"] / args.steps, 2) for n, v in kt.items()},
                     "kernel_GBps": {n: round(v["model_bytes"] / (v["total_ms"] * 1e-3) / 1e9, 1)
                                     for n, v in kt.items() if v["total_ms"] > 0}}
        if rr.get("kt_iso"):
            ki = rr["kt_iso"]
            dst[mode.replace("_paper", "")]["isolated"] = {
                "kernel_ms": {n: round(v["total_ms"], 2) for n, v in ki.items()},
                "kernel_GBps": {n: round(v["model_bytes"] / (v["total_ms"] * 1e-3) / 1e9, 1)
                                for n, v in ki.items() if v["total_ms"] > 0},
                "how": "batched launches of the one-after-the-other Lanczos and projection pass"}
    out.update(extras)
    if model:
        out["model_operator"] = {"chi0_applies_per_s": round(n_apply / model, 2), "step_s": round(model, 4),
                                 "how": "the same 64-step Lanczos + 32-frequency projection on eps~ - 1, the "
                                        "model operator of Sec. V (H -> T: one diagonal division per band "
                                        "solve), FP64"}
    rr = r.get("rec")
    if rr:
        lz = r["lanczos_s"] or None
        out["recycling"] = {
            "imaginary_frequencies": rr["n_w"], "lanczos_steps": rr["k"],
            "lanczos_plus_recycle_s": round(rr["seconds"], 4),
            "recycle_s": round(rr["seconds"] - lz, 4) if lz else None,
            "E_rel_dev_vs_direct": {"max": float(max(rr["dev"])), "w0": float(rr["dev"][0]),
                                    "last": float(rr["dev"][-1])},
            "how": "lgw_lanczos_recycle (static Lanczos + one small basis per band, Sec. VI) at the "
                   "imaginary frequencies of the step, against the step's directly projected E(z) "
                   "on the same basis; recycle_s subtracts the sequential Lanczos time"}
    pm = "fp64" if "fp64" in results else ("fp64_paper" if "fp64_paper" in results else None)
    if pm:
        out["plain_fp64"] = {"chi0_applies_per_s": round(results[pm]["plain"], 2),
                             "sample": "one chi0 apply (1 column, 1 frequency) per call, FP64 "
                                       + ("(same solver form as the headline)" if pm == "fp64"
                                          else "(unpreconditioned form)")
                                       + ": 2 columns x z = 0, 0.13i, 2i, 0.5+0.1eV*i",
                             "value_over_plain": round(value / results[pm]["plain"], 2)}
    if "fp64" in results and "fp64_paper" in results:
        f, p_ = results["fp64"], results["fp64_paper"]
        out["fast_vs_paper_fp64"] = {
            "alpha_rel": float(np.abs(f["alpha"] - p_["alpha"]).max() / np.abs(p_["alpha"]).max()),
            "beta_rel": float(np.abs(f["beta"] - p_["beta"]).max() / np.abs(p_["alpha"]).max()),
            "E_rel": float(max(np.linalg.norm(f["E"][i] - p_["E"][i]) / np.linalg.norm(p_["E"][i])
                               for i in range(len(zs)))),
            "speedup": round(p_["elapsed"] / f["elapsed"], 3)}
    if "fp64" in results and "mixed" in results:
        f, m = results["fp64"], results["mixed"]
        Em = m["E_fp64_basis"]
        out["mixed_vs_fp64"] = {
            "alpha_rel": float(np.abs(m["alpha"] - f["alpha"]).max() / np.abs(f["alpha"]).max()),
            "beta_rel": float(np.abs(m["beta"] - f["beta"]).max() / np.abs(f["alpha"]).max()),
            "E_rel_same_basis": float(max(np.linalg.norm(Em[i] - f["E"][i]) / np.linalg.norm(f["E"][i])
                                          for i in range(len(zs)))),
            "speedup": round(f["elapsed"] / m["elapsed"], 3),
            "mixed_solve_tol": args.mixed_tol, "target": 1e-6}
        g = out["mixed_vs_fp64"]
        g["within_target"] = bool(max(g["alpha_rel"], g["beta_rel"], g["E_rel_same_basis"]) <= 1e-6)
    if not args.no_cpu:
        cores = cpu_cores()
        # two columns per core (the first is the sampled accuracy check), each
        # at the four sample frequencies: about 10 s of wall time
        xs = [x_s] + list(random_potentials(w.N, 2 * cores - 1, (14083036, 2, 0, 9)))
        res, wall, busy = cpu_baseline(w, z_s, xs, cores)
        n_cpu = len(xs) * len(z_s)
        out["cpu_baseline"] = {"value": round(n_cpu / wall, 4), "unit": "chi0-applies/s",
                               "cores": min(cores, len(xs)), "kind": "oracle",
                               "cpu_model": cpu_model(),
                               "sample": f"matrix-free FP64 Sternheimer oracle (numpy FFT, SciPy "
                                         f"CG/GMRES) on {len(xs)} columns x z = 0, 0.13i, 2i, "
                                         f"0.5+0.1eV*i of the same workload ({n_cpu} chi0 applies), "
                                         f"one column per task over {min(cores, len(xs))} single-threaded "
                                         f"worker processes: {wall:.1f}s wall, {busy:.1f}s summed"}
        ref = res[0]
        out["oracle_check"] = {mode: float(max(np.linalg.norm(rr["dn_s"][i] - ref[i]) /
                                               np.linalg.norm(ref[i]) for i in range(len(z_s))))
                               for mode, rr in results.items()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
