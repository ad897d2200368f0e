"""Benchmark of the reconstruction hot path on one MI355X.

A step is one full reconstruction (recon_solve: input conditioning, 10 outer
steps of deformed-mesh mass, limited source, multigrid-preconditioned solve,
step control, and the output delta_r) of the 512^3 lognormal field
(box 1000 Mpc/h, sigma_g = 2.0), with the density already resident in HBM.
The headline value is the wall time of the mixed-precision solve (FP32
V-cycle inside the FP64 Krylov loop); the FP64 solve is timed the same way
and both are compared (rel. L2 of phi and delta_r).  The finest-level
red-black Gauss-Seidel smoother is timed live with hipEvents inside the
library (cfg.profile) to give its achieved HBM bandwidth.

Prints one JSON line.  --gpus N > 1 is not supported: the library runs one
GPU per process, and a split of the grid into i-slabs over several GPUs
(one-plane halo exchanges per sweep, scalar all-reduces per Krylov step) is
not built.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
METRIC = "recon wall time + smoother HBM GB/s at 512^3, mixed vs FP64, at 1e-6 rel L2"


# The finest-level sweep kernels (the instantiation that reads u, a and b).
FUSED_KERNEL = {"mixed": "k_rbgs_fused<float,8,0,{0,1},128,256,2,4,0,1>",
                "fp64": "k_rbgs_fused<double,16,0,{0,1},64,512,2,6,0,1>"}
COUNTERS = os.path.join(ROOT, "profiles", "rbgs_fused_512_counters.json")


def measured_traffic(kernel, n):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE and
    WRITE_SIZE counter runs (scaled by the same counters on a plain 1 GiB
    copy), or None when they are absent, were taken at another size, or the
    kernel source has changed since."""
    import hashlib
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
        h = hashlib.sha256()
        for src in c["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        digest = h.hexdigest()
    except (OSError, ValueError, KeyError):
        return None
    if digest != c["source_sha256"] or c["n"] != n or kernel not in c["kernels"]:
        return None
    return int(round(c["kernels"][kernel]["traffic_bytes"]))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(rho, n, stats, cores, workload):
    """Oracle (FP64 C, OpenMP) on a bounded sample of the same workload, timed
    on this host: the first outer step's own code path at full size -- the
    deformed-mesh mass, the source, the oracle's Krylov solve capped at one
    and at two V-cycles (the difference is one Krylov iteration: V-cycle,
    operator, dot products and vector updates; the rest is the solve's
    set-up, coefficient hierarchy and true residual) and the step control --
    scaled by the GPU solve's outer steps and V-cycle count.  Beside it, the
    oracle's full solve of this workload as recorded when its golden values
    were written (threads stated there)."""
    import oracle

    oracle.build(force=False)
    m = oracle.normalize(rho)
    phi = np.zeros_like(m)
    t0 = time.perf_counter()
    M = oracle.meshmass(phi, m)
    t_mm = time.perf_counter() - t0
    t0 = time.perf_counter()
    b = oracle.source(phi, M)
    t_src = time.perf_counter() - t0
    del m
    t_solve = {}
    u = None
    for k in (1, 2):
        cfg = oracle.Config(max_vcycles=k, tol=1e-300)
        t0 = time.perf_counter()
        try:
            u, _, _ = oracle.mg_solve(M, b, cfg)
        except oracle.OracleError as e:  # capped: no convergence, by design
            assert e.code == -4
        t_solve[k] = time.perf_counter() - t0
    t_iter = t_solve[2] - t_solve[1]
    t_setup = max(t_solve[1] - t_iter, 0.0)
    dphi = oracle.smooth(b)  # an increment of the solve's shape, for the step control's timing
    t0 = time.perf_counter()
    oracle.choose_step(phi, dphi, oracle.Config())
    t_step = time.perf_counter() - t0
    outer = stats["outer_steps"]
    vc = stats["vcycles_total"]
    est = outer * (t_mm + t_src + t_setup + t_step) + vc * t_iter
    out = {"value": round(est, 3), "unit": "s", "cores": cores, "kind": "oracle",
           "sample": ("the oracle's first outer step at %d^3 on this host: meshmass %.2fs, source %.2fs, Krylov "
                      "solve capped at 1 / 2 V-cycles %.2fs / %.2fs (one iteration %.2fs, set-up and true residual "
                      "%.2fs), step control %.2fs; scaled by the GPU solve's %d outer steps and %d V-cycles"
                      % (n, t_mm, t_src, t_solve[1], t_solve[2], t_iter, t_setup, t_step, outer, vc))}
    gold = oracle_samples(workload)
    if gold is not None and "oracle_seconds" in gold:
        out["full_solve_recorded"] = {"value": gold["oracle_seconds"], "unit": "s", "threads": gold.get("threads"),
                                      "source": "tests/golden/%s_oracle_forward.json (the whole 10-step solve, "
                                                "timed when the golden values were written)" % workload}
    return out


def oracle_samples(workload):
    """The FP64 oracle's solve of this workload at 2048 seeded voxels, stored
    by the tests' golden-value script (None if not stored)."""
    path = os.path.join(ROOT, "tests", "golden", workload + "_oracle_forward.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


PROBE_LIB = os.path.join(ROOT, "paper_1611_09638_amd", "libstream_probe.so")
PROBE_KINDS = {"read": (0, 1), "write": (1, 1), "copy": (2, 2), "three_reads_one_write": (3, 4)}


def _probe_lib():
    import ctypes
    if not os.path.exists(PROBE_LIB):
        raise RuntimeError("%s is not built (run __graft_entry__.build())" % PROBE_LIB)
    L = ctypes.CDLL(PROBE_LIB)
    vp = ctypes.c_void_p
    L.stream_probe_run.restype = ctypes.c_int
    L.stream_probe_run.argtypes = [ctypes.c_int, vp, vp, vp, vp, ctypes.c_size_t, ctypes.c_int, vp, ctypes.c_int,
                                   vp, ctypes.POINTER(ctypes.c_float)]
    return L


def stream_ceilings(torch, dev, reps=5, gib=4, kinds=None):
    """Achievable HBM bandwidth on this GPU for the access patterns of the
    path, from the hand-written streaming probes (libstream_probe.so: 16-byte
    accesses, every byte moved once) over arrays of `gib` GiB each (FP32),
    far beyond the 256 MB last-level cache: read only, write only, copy
    (1 read, 1 write) and 3 reads + 1 write (the smoother's mix).  GB/s =
    bytes moved / mean kernel time (hipEvents); the best over grid sizes
    (down to one vector per thread) and cache policies (plain, nontemporal)."""
    import ctypes
    L = _probe_lib()
    nbytes = gib << 30
    nel = nbytes // 4
    blocks = (16384, 65536, nbytes // (16 * 256))
    arrs = [torch.ones(nel, device=dev) for _ in range(4)]
    part = torch.empty(max(blocks), device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    out = {}
    for name, (kind, arrays) in PROBE_KINDS.items():
        if kinds and name not in kinds:
            continue
        best = None
        for nt in (0, 16):
            for nb in blocks:
                ms = ctypes.c_float(0.0)
                rc = L.stream_probe_run(kind | nt, arrs[0].data_ptr(), arrs[1].data_ptr(), arrs[2].data_ptr(),
                                        arrs[3].data_ptr(), nbytes, nb, part.data_ptr(), reps, stream,
                                        ctypes.byref(ms))
                if rc:
                    raise RuntimeError("stream probe %s failed (%d)" % (name, rc))
                gbs = arrays * nbytes / (ms.value * 1e-3) / 1e9
                if best is None or gbs > best[0]:
                    best = (gbs, nb, nt)
        out[name + "_GBps"] = round(best[0], 1)
        out[name + "_how"] = "%d blocks%s" % (best[1], ", nontemporal" if best[2] else "")
    out["array_GiB"] = gib
    del arrs, part
    torch.cuda.empty_cache()
    return out


def particle_bench(torch, binding, inputs, args):
    """512^3 Zel'dovich particles (1000 Mpc/h, rms displacement 1.5 cells, seed
    5), mixed precision: particles assigned to the grid once (the default) and
    deposited at their Lagrangian positions every step; wall time, steps, and
    the correlation of the two delta_r; then the reverse mode of the latter
    (forward with a tape, and the gradient with respect to the positions)."""
    n, box = 512, 1000.0
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    pos = torch.from_numpy(inputs.zeldovich_particles(n, box, 1.5, 5)).to(dev)
    log("particles generated in %.1fs" % (time.perf_counter() - t0))
    out = {"workload": "zeldovich512", "n": n, "box": box, "rms_cells": 1.5, "particles": n ** 3,
           "precision": "mixed", "steps": args.steps}
    res = {}
    for mode in (0, 1):
        rec = binding.Recon(n, binding.Config(precision=binding.MIXED, particle_deposit=mode), device=dev)
        for _ in range(args.warmup):
            rec.solve_particles(pos, box, want_phi=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, d, st = rec.solve_particles(pos, box, want_phi=False)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        key = "deposit_each_step" if mode else "grid_once"
        out[key] = {"wall_s": round(wall, 4), "vcycles_total": st["vcycles_total"], "alpha": st["alpha"],
                    "rms_sigma_first": st["rms_sigma"][0], "rms_sigma_last": st["rms_sigma"][-1],
                    "mean_M_last": st["kappa"][-1]}
        res[mode] = d.double()
        log("%s: %.3f s" % (key, wall))
        del rec
        torch.cuda.empty_cache()
    out["corr_delta_r"] = float(torch.corrcoef(torch.stack([res[0].flatten(), res[1].flatten()]))[0, 1])
    # reverse mode of the deposit-each-step solve: dL/d(positions) for a
    # random linear loss on delta_r, with an FP64 tape
    rec = binding.Recon(n, binding.Config(precision=binding.MIXED, particle_deposit=1, record_tape=1), device=dev)
    gd = torch.randn((n, n, n), dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(7))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rec.solve_particles(pos, box, want_phi=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g = rec.backward_particles(pos, gd)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out["reverse_mode"] = {"forward_with_tape_s": round(t1 - t0, 4), "backward_s": round(t2 - t1, 4),
                           "grad_rms": float(g.pow(2).mean().sqrt()), "grad_finite": bool(torch.isfinite(g).all())}
    log("particle reverse mode: forward %.3f s, backward %.3f s" % (t1 - t0, t2 - t1))
    del rec, g
    torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


# The workloads of the paper-shaped configurations: name, workload, solver
# settings, precisions, and whether the reverse mode is timed as well.  The
# 128^3 adjoint case uses the tolerance its oracle gradient was computed with.
CONFIG_RUNS = [
    ("cfg1", "zeldovich32", dict(coarse_n=8, max_outer=10), ("fp64", "mixed"), False),
    ("cfg2", "lognormal256", {}, ("fp64", "mixed"), False),
    ("cfg3", "lognormal512", {}, ("fp64", "mixed"), False),
    ("cfg4", "lognormal128", dict(tol=1e-13, max_vcycles=400), ("fp64",), True),
]


def _loss_window(torch, n, box, dev, R=10.0):
    """exp(-k^2 R^2) on the FFT grid: the filtered-power loss of the 128^3
    adjoint case, whose gradient with respect to delta_r is
    2 n^3 Re(ifftn(W fftn(delta_r)))."""
    k = 2 * np.pi * np.fft.fftfreq(n, box / n)
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    return torch.from_numpy(np.exp(-k2 * R ** 2)).to(dev)


def configs_bench(torch, binding, inputs, args):
    """GPU wall time of every paper-shaped configuration that fits the
    oracle's reach (32^3 particles, 256^3, 512^3 and 128^3 densities): the
    median of --steps solves after --warmup, inputs resident in HBM; for the
    128^3 case also the reverse mode over the recorded tape.  The 1024^3
    particle case is timed by its own test (its inputs take minutes to
    generate).  Beside each, the oracle's whole solve as recorded with its
    golden values, and for the 32^3 case the oracle timed here, on all host
    threads and on one."""
    dev = torch.device("cuda:0")
    out = {"configs": [], "steps": args.steps, "warmup": args.warmup}
    prec = {"fp64": binding.FP64, "mixed": binding.MIXED}
    for name, wl, extra, precs, adjoint in CONFIG_RUNS:
        w = inputs.WORKLOADS[wl]
        n, box = w["n"], w["box"]
        kind, arr, _, _ = inputs.make_workload(wl)
        x = torch.from_numpy(arr).to(dev)
        row = {"name": name, "workload": wl, "n": n, "box": box, "input": kind, "settings": extra, "gpu": {}}
        for pn in precs:
            rec = binding.Recon(n, binding.Config(precision=prec[pn], record_tape=1 if adjoint else 0, **extra),
                                device=dev)
            solve = rec.solve_particles if kind == "particles" else rec.solve
            for _ in range(args.warmup):
                solve(x, box, want_phi=False)
            walls, bw = [], []
            gd = None
            for _ in range(args.steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, d, st = solve(x, box, want_phi=False)
                torch.cuda.synchronize()
                walls.append(time.perf_counter() - t0)
                if adjoint:
                    if gd is None:
                        gd = (2.0 * n ** 3 * torch.fft.ifftn(_loss_window(torch, n, box, dev) *
                                                              torch.fft.fftn(d)).real).contiguous()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    rec.backward(gd)
                    torch.cuda.synchronize()
                    bw.append(time.perf_counter() - t0)
            r = {"wall_s": round(float(np.median(walls)), 4), "vcycles_total": st["vcycles_total"],
                 "outer_steps": st["outer_steps"]}
            if adjoint:
                r["backward_s"] = round(float(np.median(bw)), 4)
            row["gpu"][pn] = r
            log("%s %s %s: %s" % (name, wl, pn, r))
            del rec
            torch.cuda.empty_cache()
        gold = oracle_samples(wl)
        if gold is not None and "oracle_seconds" in gold:
            row["oracle_recorded"] = {"seconds": gold["oracle_seconds"], "threads": gold.get("threads"),
                                      "source": "tests/golden/%s_oracle_forward.json" % wl}
        out["configs"].append(row)
        del x
    if not args.skip_cpu:
        out["oracle_cfg1"] = configs_cpu_baseline(inputs, ("cfg1",))["cfg1"]
    print(json.dumps(out), flush=True)


def configs_cpu_baseline(inputs, names):
    """The oracle (FP64 C with OpenMP) timed on this host for the named
    configurations: its whole forward solve, and for the 128^3 adjoint case
    the reverse mode too, on all host threads (OMP_NUM_THREADS, else every
    core); the 32^3 case also on one thread, in a child process that sets
    OMP_NUM_THREADS=1 before the oracle library is loaded."""
    import subprocess
    import oracle
    oracle.build(force=False)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))
    res = {}
    for name, wl, extra, _, adjoint in CONFIG_RUNS:
        if name not in names:
            continue
        w = inputs.WORKLOADS[wl]
        n, box = w["n"], w["box"]
        kind, arr, _, _ = inputs.make_workload(wl)
        rho = oracle.cic_particles(arr, n, box) if kind == "particles" else arr
        cfg = oracle.Config(record_tape=1 if adjoint else 0, **extra)
        t0 = time.perf_counter()
        _, d, st = oracle.solve(rho, box, cfg)
        r = {"threads": threads, "forward_s": round(time.perf_counter() - t0, 3), "vcycles_total": sum(st["vcycles"])}
        if adjoint:
            k = 2 * np.pi * np.fft.fftfreq(n, box / n)
            k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
            gd = 2.0 * n ** 3 * np.real(np.fft.ifftn(np.exp(-k2 * 100.0) * np.fft.fftn(d)))
            t0 = time.perf_counter()
            oracle.backward(gd, None, box, cfg)
            r["backward_s"] = round(time.perf_counter() - t0, 3)
        if name == "cfg1" and threads > 1:
            env = dict(os.environ, OMP_NUM_THREADS="1")
            cp = subprocess.run([sys.executable, os.path.abspath(__file__), "--configs-oracle", "cfg1"], env=env,
                                capture_output=True, text=True, check=True)
            r["one_thread"] = json.loads(cp.stdout.strip().splitlines()[-1])["cfg1"]
        res[name] = r
        log("oracle %s: %s" % (name, r))
    return res


def quality_bench(torch, binding, inputs):
    """Sec. III on stand-in data: Zel'dovich inputs at 256^3 (600 Mpc/h, cells of
    2.34 Mpc/h) with the linear density -div Psi known exactly.  The cross-
    correlation r(k) and the propagator C(k) of the nonlinear (CIC) and the
    reconstructed density with the linear field (mixed precision), for rms
    displacements of 1.5 and 3.5 cells; on the 3.5-cell input (where the
    compression limiter engages) with 20 outer steps, the sweeps xi_m in (1/5,
    1/10, 1/20) at v_m = 10 and v_m in (5, 10, 20) at xi_m = 1/10 (App. B).
    The library's options are compared on the same inputs: the exact-Jacobian
    solve, the particles deposited at their Lagrangian positions (alone and
    with the exact Jacobian) and the paper's mass update.  Diagnostics on the
    host (numpy)."""
    from paper_1611_09638_amd import diagnostics as dg
    n, box = 256, 600.0
    dev = torch.device("cuda:0")
    out = {"quality": "Zel'dovich stand-in for Sec. III", "n": n, "box": box, "precision": "mixed", "shells": 16}
    for rms in (1.5, 3.5):
        psi = inputs.zeldovich_displacement(n, box, rms, 31)
        dl = dg.linear_density(psi)
        pos = torch.from_numpy(inputs.particles_from_displacement(psi, box)).to(dev)
        del psi
        runs = [("default", {}), ("exact Jacobian", dict(full_operator=1)),
                ("particle deposit", dict(particle_deposit=1)),
                ("particle deposit + exact Jacobian", dict(particle_deposit=1, full_operator=1)),
                ("mass update", dict(mass_update=1))]
        if rms == 3.5:
            runs = [("xi_m=%g" % x, dict(xi_m=x, max_outer=20)) for x in (0.2, 0.1, 0.05)]
            runs += [("v_m=%g" % v, dict(v_m=v, max_outer=20)) for v in (5.0, 20.0)]
            runs += [("xi_m=0.1,10 steps", {}), ("exact Jacobian, 20 steps", dict(full_operator=1, max_outer=20)),
                     ("particle deposit, 20 steps", dict(particle_deposit=1, max_outer=20))]
        rec = binding.Recon(n, binding.Config(precision=binding.MIXED), device=dev)
        nl = dg.propagator(rec.cic(pos, box).cpu().numpy() - 1.0, dl, box, 16)
        del rec
        block = {"k": [round(x, 4) for x in nl["k"]], "nonlinear": {"r": [round(x, 4) for x in nl["r"]],
                                                                   "C": [round(x, 4) for x in nl["C"]]}}
        for label, kw in runs:
            rec = binding.Recon(n, binding.Config(precision=binding.MIXED, **kw), device=dev)
            t0 = time.perf_counter()
            try:
                _, dr, st = rec.solve_particles(pos, box, want_phi=False)
            except binding.ReconError as e:
                block[label] = {"error": str(e)}
                log("rms %.1f %s: %s" % (rms, label, e))
                del rec
                torch.cuda.empty_cache()
                continue
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            q = dg.propagator(dr.cpu().numpy(), dl, box, 16)
            block[label] = {"r": [round(x, 4) for x in q["r"]], "C": [round(x, 4) for x in q["C"]],
                            "wall_s": round(wall, 3), "outer_steps": st["outer_steps"],
                            "rms_sigma_last": st["rms_sigma"][-1], "min_lambda0": st["min_lambda0"],
                            "alpha_last": st["alpha"][-3:]}
            log("rms %.1f %s: %.2f s, rms(Sigma) %.3g" % (rms, label, wall, st["rms_sigma"][-1]))
            del rec
            torch.cuda.empty_cache()
        out["rms_%g_cells" % rms] = block
    print(json.dumps(out), flush=True)


def mass_update_bench(torch, binding, inputs, args):
    """Mixed solves of lognormal512_mild with M gathered by CIC every step and
    with the paper's mass update, and the time of the update's two passes
    (K = M e^-1: read phi, M, write six fields; the streaming 19-point
    application: read the six fields and f, write the change): 64 + 64
    algorithmic B/node."""
    name = "lognormal512_mild"
    w = inputs.WORKLOADS[name]
    n, box = w["n"], w["box"]
    rho = inputs.lognormal_density(n, box, w["sigma_g"], w["seed"])
    dev = torch.device("cuda:0")
    rho_d = torch.from_numpy(rho).to(dev)
    out = {"workload": name, "n": n, "box": box, "sigma_g": w["sigma_g"], "precision": "mixed", "steps": args.steps}
    res = {}
    for mode in (0, 1):
        rec = binding.Recon(n, binding.Config(precision=binding.MIXED, mass_update=mode), device=dev)
        for _ in range(args.warmup):
            rec.solve(rho_d, box)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            phi, delta, st = rec.solve(rho_d, box)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        key = "mass_update" if mode else "cic_gather"
        out[key] = {"wall_s": round(wall, 4), "vcycles_total": st["vcycles_total"], "alpha": st["alpha"],
                    "rms_sigma_first": st["rms_sigma"][0], "rms_sigma_last": st["rms_sigma"][-1],
                    "mean_M_last": st["kappa"][-1]}
        res[mode] = (phi, delta)
        log("%s: %.3f s, %d V-cycles" % (key, wall, st["vcycles_total"]))
        if mode == 1:
            h = box / n
            phi_g = (phi / (h * h)).contiguous()
            f = phi_g.clone()
            rec.mass_change(phi_g, rho_d, f)  # warm
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 10
            e0.record()
            for _ in range(reps):
                rec.mass_change(phi_g, rho_d, f)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            gbs = 128 * n ** 3 / (ms * 1e-3) / 1e9
            out["mass_change_kernels"] = {"ms": round(ms, 3), "alg_bytes_per_node": 128, "GBps": round(gbs, 1),
                                          "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
                                          "note": "K = M e^-1 (gather) and the streaming 19-point application, once per outer step"}
        del rec
        torch.cuda.empty_cache()
    d0, d1 = (res[m][1].double() for m in (0, 1))
    out["rel_l2_delta_r_update_vs_gather"] = float(torch.linalg.norm(d1 - d0) / torch.linalg.norm(d0))
    out["corr_delta_r_update_vs_gather"] = float(torch.corrcoef(torch.stack([d0.flatten(), d1.flatten()]))[0, 1])
    print(json.dumps(out), flush=True)


def full_operator_bench(torch, binding, inputs, args):
    """Mixed solves of the workload with the x ~ xi operator and with the
    exact-Jacobian operator in the Krylov loop (full_operator = 1): wall time,
    V-cycles and rms(Sigma) per step.  The full operator's kernels are timed
    from a kernel trace of this run: the Krylov product q = L_K p with p.q
    reads six K fields and p and writes q (64 algorithmic B/node), the Krylov
    residual reads six K fields, u and b and writes r and its FP32 copy
    (76 B/node)."""
    name = args.workload
    w = inputs.WORKLOADS[name]
    n, box = w["n"], w["box"]
    rho = inputs.lognormal_density(n, box, w["sigma_g"], w["seed"])
    dev = torch.device("cuda:0")
    rho_d = torch.from_numpy(rho).to(dev)
    out = {"workload": name, "n": n, "box": box, "sigma_g": w["sigma_g"], "precision": "mixed", "steps": args.steps}
    for mode in (0, 1):
        rec = binding.Recon(n, binding.Config(precision=binding.MIXED, full_operator=mode), device=dev)
        for _ in range(args.warmup):
            rec.solve(rho_d, box)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            phi, delta, st = rec.solve(rho_d, box)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        key = "full_operator" if mode else "x_approx_xi"
        out[key] = {"wall_s": round(wall, 4), "vcycles": st["vcycles"], "vcycles_total": st["vcycles_total"],
                    "alpha": st["alpha"], "rms_sigma": [round(x, 5) for x in st["rms_sigma"]],
                    "min_lambda0": st["min_lambda0"]}
        log("%s: %.3f s, %d V-cycles, rms(Sigma) %.4f" % (key, wall, st["vcycles_total"], st["rms_sigma"][-1]))
        del rec
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lognormal512")
    ap.add_argument("--skip-cpu", action="store_true", help="omit the oracle CPU baseline")
    ap.add_argument("--only", choices=["both", "mixed", "fp64"], default="both")
    ap.add_argument("--probe", action="store_true",
                    help="counter run: one plain 1 GiB copy (calibration) and one fused sweep per precision at 512^3")
    ap.add_argument("--stream", action="store_true", help="only the streaming-bandwidth ceilings of this GPU")
    ap.add_argument("--quality", action="store_true",
                    help="the paper's quality measures (Sec. III) on Zel'dovich inputs at 256^3: r(k) and the "
                         "propagator of the nonlinear and reconstructed fields, and the xi_m / v_m sweeps")
    ap.add_argument("--particle-deposit", action="store_true",
                    help="particles deposited at their Lagrangian positions every step against one CIC onto the "
                         "grid, on 512^3 Zel'dovich particles, mixed precision")
    ap.add_argument("--full-operator", action="store_true",
                    help="the exact-Jacobian operator in the linear solve against x ~ xi on --workload (mixed)")
    ap.add_argument("--configs", action="store_true",
                    help="GPU wall time of the paper-shaped configurations (32^3 particles, 256^3, 512^3, 128^3 "
                         "with its reverse mode) beside the oracle's recorded and measured times")
    ap.add_argument("--configs-oracle", nargs="+", metavar="CFG",
                    help="the oracle alone on this host's cores for the named configurations (no GPU used)")
    ap.add_argument("--mass-update", action="store_true",
                    help="the paper's mass update (App. A) against the per-step CIC gather on lognormal512_mild, "
                         "mixed precision, and the bandwidth of its two kernels")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU (one process per GPU); --gpus %d is not supported: "
              "the multi-GPU slab decomposition is not built" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.configs_oracle:
        from paper_1611_09638_amd import inputs
        print(json.dumps(configs_cpu_baseline(inputs, tuple(args.configs_oracle))), flush=True)
        return

    import torch

    from paper_1611_09638_amd import binding, inputs

    if args.stream:
        print(json.dumps({"stream": stream_ceilings(torch, torch.device("cuda:0"), reps=10)}), flush=True)
        return

    if args.probe:
        n = 512
        dev = torch.device("cuda:0")
        g = torch.Generator(device=dev).manual_seed(0)
        a = torch.rand((n, n, n), dtype=torch.float64, device=dev, generator=g) + 0.01
        u = torch.rand((n, n, n), dtype=torch.float64, device=dev, generator=g)
        b = torch.rand((n, n, n), dtype=torch.float64, device=dev, generator=g)
        # calibration: the hand-written copy probe over 4 GiB (4 GiB read +
        # 4 GiB written per launch, far beyond the last-level cache)
        import ctypes
        x = torch.ones(1 << 30, device=dev)
        y = torch.empty_like(x)
        ms = ctypes.c_float(0.0)
        rc = _probe_lib().stream_probe_run(2, y.data_ptr(), x.data_ptr(), None, None, 4 << 30, 8192, None, 1,
                                           torch.cuda.current_stream(dev).cuda_stream, ctypes.byref(ms))
        assert rc == 0
        del x, y
        torch.cuda.synchronize()
        rec = binding.Recon(n, binding.Config(precision=binding.MIXED), device=dev)
        rec.rbgs(u.float(), a.float(), b.float(), first=1, variant=2)
        rec.rbgs(u, a, b, first=1, variant=2)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "copy 4 GiB (twice: untimed + timed) + fused sweep f32 + fused sweep f64",
                          "n": n, "copy_bytes_read": 4 << 30, "copy_bytes_written": 4 << 30,
                          "sweep_alg_bytes_f32": 16 * n ** 3, "sweep_alg_bytes_f64": 32 * n ** 3}), flush=True)
        return

    if args.mass_update:
        mass_update_bench(torch, binding, inputs, args)
        return
    if args.full_operator:
        full_operator_bench(torch, binding, inputs, args)
        return
    if args.quality:
        quality_bench(torch, binding, inputs)
        return
    if args.configs:
        configs_bench(torch, binding, inputs, args)
        return
    if args.particle_deposit:
        particle_bench(torch, binding, inputs, args)
        return

    w = inputs.WORKLOADS[args.workload]
    if w["kind"] != "lognormal":
        raise SystemExit("bench workload must be a density grid")
    n, box = w["n"], w["box"]
    t0 = time.perf_counter()
    rho = inputs.lognormal_density(n, box, w["sigma_g"], w["seed"])
    log("input %s generated in %.1fs" % (args.workload, time.perf_counter() - t0))
    dev = torch.device("cuda:0")
    stream = stream_ceilings(torch, dev)
    log("stream ceilings %s" % stream)
    rho_d = torch.from_numpy(rho).to(dev)

    results = {}
    modes = {"fp64": binding.FP64, "mixed": binding.MIXED}
    if args.only != "both":
        modes = {args.only: modes[args.only]}
    for name, prec in modes.items():
        rec = binding.Recon(n, binding.Config(precision=prec, profile=1), device=dev)
        for i in range(args.warmup):
            rec.solve(rho_d, box)
            log("%s warmup %d done" % (name, i))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        walls, sts = [], []
        for i in range(args.steps):
            phi, delta, st = rec.solve(rho_d, box)
            walls.append(st["ms_total"])
            sts.append(st)
            log("%s step %d: %.1f ms, %d V-cycles" % (name, i, st["ms_total"], st["vcycles_total"]))
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        results[name] = dict(wall_s=wall, ms=float(np.median(walls)), stats=sts[-1], phi=phi, delta=delta)
        del rec
        torch.cuda.empty_cache()

    head = "mixed" if "mixed" in results else "fp64"
    H = results[head]
    st = H["stats"]
    node_bytes = 16 if head == "mixed" else 32
    sweep_ms = st["smoother_ms"] / max(st["smoother_sweeps"], 1)
    achieved = node_bytes * n ** 3 / (sweep_ms * 1e-3) / 1e9
    kernel = FUSED_KERNEL[head]
    out = {
        "metric": METRIC,
        "value": round(H["wall_s"], 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(H["wall_s"] * 1e3, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "box": box, "sigma_g": w["sigma_g"], "seed": w["seed"],
                   "max_outer": 10, "tol": 1e-10, "solver": "pcg+vcycle(2,2)", "precision": head},
        "outer_steps": st["outer_steps"],
        "vcycles_total": st["vcycles_total"],
        "vcycles": st["vcycles"],
        "alpha": st["alpha"],
        "alpha_limit": st["alpha_limit"],
        "rms_sigma": [float("%.6g" % x) for x in st["rms_sigma"]],
    }
    for name, R in results.items():
        s = R["stats"]
        nb = 16 if name == "mixed" else 32
        sm = s["smoother_ms"] / max(s["smoother_sweeps"], 1)
        out["%s_s" % name] = round(R["wall_s"], 4)
        zm = s["smoother_zero_ms"] / max(s["smoother_zero_sweeps"], 1)
        fm = s["smoother_folded_ms"] / max(s["smoother_folded_sweeps"], 1)
        # the folded sweep also reads the coarse correction (1/8 of a field)
        fb = nb + nb / 4 / 8
        out["%s_smoother" % name] = {"sweeps": s["smoother_sweeps"], "ms_per_sweep": round(sm, 4),
                                     "GBps": round(nb * n ** 3 / (sm * 1e-3) / 1e9, 1),
                                     "bytes_per_node": nb,
                                     "zero_start_sweeps": s["smoother_zero_sweeps"],
                                     "zero_start_ms_per_sweep": round(zm, 4),
                                     "zero_start_GBps": round(nb * 3 // 4 * n ** 3 / (zm * 1e-3) / 1e9, 1),
                                     "folded_sweeps": s["smoother_folded_sweeps"],
                                     "folded_ms_per_sweep": round(fm, 4),
                                     "folded_bytes_per_node": fb,
                                     "folded_GBps": round(fb * n ** 3 / (fm * 1e-3) / 1e9, 1),
                                     "vcycles": s["vcycles_total"]}
    gold = oracle_samples(args.workload)
    if gold is not None:
        vox = torch.tensor(gold["voxels"], device=dev)
        for name, R in results.items():
            cmp = {"alpha_equal": R["stats"]["alpha"] == gold["alpha"]}
            for key, f in (("phi", R["phi"]), ("delta_r", R["delta"])):
                g = torch.tensor(gold[key], dtype=torch.float64, device=dev)
                cmp["rel_l2_" + key] = float((f.reshape(-1)[vox] - g).norm() / g.norm())
            out["%s_vs_oracle" % name] = cmp
    if len(results) == 2:
        a, b = results["mixed"], results["fp64"]
        out["speedup_mixed_vs_fp64"] = round(b["wall_s"] / a["wall_s"], 3)
        out["rel_l2_phi_mixed_vs_fp64"] = float((a["phi"] - b["phi"]).norm() / b["phi"].norm())
        out["rel_l2_delta_mixed_vs_fp64"] = float((a["delta"] - b["delta"]).norm() / b["delta"].norm())
        out["alpha_equal"] = a["stats"]["alpha"] == b["stats"]["alpha"]
    out["roofline"] = {"bound": "hbm", "kernel": kernel + " (finest level, one launch per sweep)",
                       "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(kernel, n),
                       "bytes_per_node_per_sweep": node_bytes, "nodes": n ** 3,
                       "algorithmic_bytes_per_launch": node_bytes * n ** 3,
                       "stream_ceiling_GBps": stream["three_reads_one_write_GBps"],
                       "frac_of_stream_ceiling": round(achieved / stream["three_reads_one_write_GBps"], 4)}
    out["stream"] = stream
    if not args.skip_cpu:
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))
        out["cpu_baseline"] = cpu_baseline(rho, n, st, cores, args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
