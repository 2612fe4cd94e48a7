"""Benchmark: lowest-32 hole eigenpairs of the DQD fin workload (256 x 48 x 48
grid, 0.4 nm, strain, B = 0.5 T along x; 3.5M complex unknowns) on one MI355X.

A step is one complete eigensolve (Lanczos bound, Chebyshev-filtered subspace
iteration with SVQB and Rayleigh-Ritz, residuals, eigenvectors returned in the
|J m_j> basis) in mixed precision -- complex FP32 filter, FP64 orthonormalisation
/ Rayleigh-Ritz / residual -- stopped at per-state residual <= 1e-5 eV.  Every
eigenvalue is compared, state by state, with the oracle's lowest 32 eigenvalues
(tests/golden, ARPACK on the assembled Hamiltonian) and must lie within 1 ueV of
it.  The plain FP64 solve at the same stopping rule is timed beside it, and a
tight FP64 solve (residual <= 1e-8 eV) is compared with the oracle as well.

value  = algorithmic H.X bytes of all stencil launches in the timed solves /
         wall time of the timed solves (GB/s, whole job, inputs resident in HBM)
roofline = the FP32 filter-step stencil (the dominant kernel): its algorithmic
         bytes per launch over its event-timed average launch duration.

Also reported (same JSON line): the device copy and triad bandwidths; the
64-Hamiltonian barrier sweep (192 x 40 x 40 each) as seconds per Hamiltonian,
batched in one hipGraph against a loop of single solves, in each precision, and
by continuation (solve_sweep); the Hellmann-Feynman backward of the 192 x 40 x 40
adjoint workload (warm time, the gradient call against its HBM roofline, error
against central finite differences); the spin-free basis, the two-hole CI, the
g-matrices and the self-consistent Schroedinger-Poisson loop; and the CPU oracle
on this host (its H.X rate, a solve time extrapolated from it, and one dense
oracle solve of the 10 x 8 x 8 workload).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra]
       python bench.py --sp-only          (only the self-consistent loop measurement)
       python bench.py --traffic-from FETCH_CSV WRITE_CSV --stencil S --nb NB --bench-log LOG
           (writes the HBM traffic summary of the FP32 stencil from two rocprofv3
           --pmc runs of `bench.py --copy-calibration --no-cpu --no-extra --steps 1
           --warmup 0 --stencil S --nb NB`, LOG the stdout of the first)
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

METRIC = "H·X GB/s; s per lowest-32-eigenpair solve, FP32-mixed vs FP64 at 1 µeV"
WORKLOAD = "dqd_256x48x48"
HBM_PEAK_GBPS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


TRAFFIC_JSON = os.path.join(ROOT, "profiles", "stencil_fp32_dqd_256x48x48_traffic.json")
STENCIL_SRC = os.path.join(ROOT, "paper_2607_08447_amd", "csrc", "stencil.hip")


def _src_hash():
    with open(STENCIL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _shape_key(tune, nb):
    return f"{tune['tile_y']},{tune['vgroup']},{tune['dma']}/nb{nb}"


def _traffic_for(kernel_src_hash, shape, alg_bytes_per_launch):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source with the
    launch shape (tile height, vector group, row DMA) and block size this run
    uses, over launches of the same average size (algorithmic bytes per launch
    within 1%: the solver's schedule decides how many vectors a launch
    filters)."""
    if not os.path.exists(TRAFFIC_JSON):
        return None
    with open(TRAFFIC_JSON) as f:
        d = json.load(f)
    if d.get("stencil_src_sha256") != kernel_src_hash:
        return None
    entry = d.get("by_launch", {}).get(shape)
    if not entry:
        return None
    alg = entry.get("algorithmic_bytes_per_launch")
    if not alg or abs(alg - alg_bytes_per_launch) > 0.01 * alg_bytes_per_launch:
        return None
    return entry.get("hbm_bytes_per_launch")


def _bench_alg_bytes(log):
    """Algorithmic bytes per FP32 stencil launch printed by a benchmark run."""
    with open(log) as f:
        for line in f:
            if line.startswith("{") and '"roofline"' in line:
                return json.loads(line)["roofline"]["algorithmic_bytes_per_launch"]
    raise SystemExit(f"{log}: no benchmark line")


def traffic_from(fetch_csv, write_csv, stencil, nb, precision="fp32", bench_log=None):
    """HBM bytes per launch of the FP32 (or FP64) stencil from rocprofv3
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) collection files.  Each
    counter is scaled by what it reads for the 1 GiB device copy the profiled
    run makes first (1 GiB read + 1 GiB written).  FP32 entries go to the JSON
    the benchmark reads, with the algorithmic bytes per launch the profiled
    benchmark run printed (bench_log, its stdout); FP64 ones are printed only."""
    import csv
    # the recurrence's steps (the benchmark's headline filter); launches without
    # an old block (product-form steps, H X) are the `void` variants
    tag = "stencil_kernel<float" if precision == "fp32" else "stencil_kernel<double"

    def per_kernel(path, counter):
        copy, sten = [], []
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                v = float(r["Counter_Value"]) * 1024.0
                name = r["Kernel_Name"]
                if "copyBuffer" in name and not copy:
                    copy.append(v)
                elif tag in name and (tag + ", void") not in name:
                    sten.append(v)
        if not copy or not sten:
            raise SystemExit(f"{path}: no copy calibration or no {precision} stencil dispatches")
        return copy[0], sten

    cf, sf = per_kernel(fetch_csv, "FETCH_SIZE")
    cw, sw = per_kernel(write_csv, "WRITE_SIZE")
    if len(sf) != len(sw):
        raise SystemExit("FETCH and WRITE runs saw different dispatch counts")
    gib = float(1 << 30)
    kf, kw = gib / cf, gib / cw
    per_launch = [kf * a + kw * b for a, b in zip(sf, sw)]
    if precision != "fp32":
        print(json.dumps({"kernel": tag, "dispatches": len(per_launch),
                          "hbm_bytes_per_launch": sum(per_launch) / len(per_launch),
                          "fetch_bytes_per_launch": kf * sum(sf) / len(sf),
                          "write_bytes_per_launch": kw * sum(sw) / len(sw),
                          "copy_calibration": {"fetch_factor": kf, "write_factor": kw}}, indent=1))
        return
    d = {}
    if os.path.exists(TRAFFIC_JSON):
        with open(TRAFFIC_JSON) as f:
            d = json.load(f)
    if d.get("stencil_src_sha256") != _src_hash():
        d = {"by_launch": {}}   # counters of an older kernel source are dropped
    d["kernel"] = ("stencil_kernel<float, ...> (FP32 Chebyshev filter step), dqd_256x48x48; "
                   "entries keyed by tile height, vector group, row DMA / block size")
    d["stencil_src_sha256"] = _src_hash()
    if bench_log is None:
        raise SystemExit("FP32 traffic needs --bench-log (the profiled run's stdout)")
    alg = _bench_alg_bytes(bench_log)
    d["by_launch"][f"{stencil}/nb{nb}"] = {
        "dispatches": len(per_launch),
        "algorithmic_bytes_per_launch": alg,
        "ratio": sum(per_launch) / len(per_launch) / alg,
        "hbm_bytes_per_launch": sum(per_launch) / len(per_launch),
        "fetch_bytes_per_launch": kf * sum(sf) / len(sf),
        "write_bytes_per_launch": kw * sum(sw) / len(sw),
        "copy_calibration": {"fetch_factor": kf, "write_factor": kw,
                             "note": "1 GiB device copy: counter bytes x factor = true bytes"},
        "made_by": [f"rocprofv3 --pmc FETCH_SIZE -- python3 bench.py --copy-calibration --no-cpu "
                    f"--no-extra --steps 1 --warmup 0 --stencil {stencil} --nb {nb}",
                    "rocprofv3 --pmc WRITE_SIZE -- (same)",
                    f"python bench.py --traffic-from <fetch csv> <write csv> --stencil {stencil} "
                    f"--nb {nb} --bench-log <stdout of the FETCH_SIZE run>"],
    }
    with open(TRAFFIC_JSON, "w") as f:
        json.dump(d, f, indent=1)
    print(json.dumps(d, indent=1))


def copy_bandwidth(torch, nbytes=2 << 30, reps=5):
    """Device-to-device copy (read + write) rate of a 2 GiB buffer, GB/s."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    dt = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    return 2.0 * nbytes / dt / 1e9


def triad_bandwidth(torch, nbytes=1 << 30, reps=5):
    """c = a + b on three 1 GiB device buffers (two streams read, one written: the
    access pattern of a filter step), GB/s counting 3 x 1 GiB per pass."""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.ones_like(a)
    c = torch.empty_like(a)
    torch.add(a, b, out=c)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.add(a, b, out=c)
    e1.record()
    e1.synchronize()
    dt = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b, c
    return 3.0 * nbytes / dt / 1e9


def _golden(tag):
    """Oracle eigenvalues stored under tests/golden (written by
    tests/golden/make_golden.py, which calls only the oracle), and the ARPACK
    operator-application count its header records, if any."""
    path = os.path.join(ROOT, "tests", "golden", f"{tag}.txt")
    matvecs, solve_s = None, None
    with open(path) as f:
        for line in f:
            if line.startswith("# matvecs"):
                matvecs = int(line.split()[2])
            if line.startswith("# oracle:") and " solve " in line:
                solve_s = float(line.split(" solve ")[1].split(" s")[0])
    return np.loadtxt(path), matvecs, solve_s


def sweep_measure(torch, hkp, workload):
    """Barrier sweep of 64 Hamiltonians (192 x 40 x 40), all to residual 1e-5 eV, in
    each precision: batched in one hipGraph-recorded solve against a loop of single
    solves over all 64 members with the same block size and stencil shape, so that
    batching and precision are measured apart; and by continuation (solve_sweep,
    mixed).  Block size and stencil launch shape are autotuned on the first member.
    Members 0, 31 and 63 of the batched mixed solve are compared with the oracle."""
    w = workload("sweep64_dqd_192x40x40")
    V = torch.from_numpy(w.V).cuda()
    S = torch.from_numpy(w.strain).cuda()
    out = {"workload": "sweep64_dqd_192x40x40", "hamiltonians": 64, "nev": w.nev,
           "stop": "per-state residual <= 1e-5 eV"}
    res = {}
    for prec in ("mixed", "fp64"):
        blk = hkp.autotune_block(V[0], w.h, w.nev, strain=S, B=w.B, candidates=[24, 32],
                                 tol=1e-5, precision=prec)
        hkp.autotune(w.shape, w.h, blk["nb"], prec)
        kw = dict(strain=S, B=w.B, nb=blk["nb"], tol=1e-5, precision=prec)
        hkp.solve_batch(V[:2], w.h, w.nev, graph=True, **kw)   # warm-up (graph recording)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rb = hkp.solve_batch(V, w.h, w.nev, graph=True, return_psi=True, **kw)
        torch.cuda.synchronize()
        t_batch = time.perf_counter() - t0
        t0 = time.perf_counter()
        E_loop, syncs_loop, st_loop = [], 0, []
        for i in range(64):
            r = hkp.solve(V[i], w.h, w.nev, return_psi=True, **kw)
            E_loop.append(r.E)
            syncs_loop += r.stats["n_host_syncs"]
            st_loop.append(r.status)
        torch.cuda.synchronize()
        t_loop = time.perf_counter() - t0
        dE = float((torch.stack(E_loop) - rb.E).abs().max())
        res[prec] = rb
        out[prec] = {"nb": blk["nb"], "nb_tuning_s": blk["seconds"],
                     "s_per_hamiltonian_batched_graph": round(t_batch / 64, 5),
                     "s_per_hamiltonian_looped": round(t_loop / 64, 5),
                     "batching_speedup": round(t_loop / t_batch, 3),
                     "batched_graph_launches": rb.stats["n_graph_launches"],
                     "batched_host_syncs": rb.stats["n_host_syncs"],
                     "batched_iterations": rb.stats["iters"],
                     "looped_host_syncs": syncs_loop,
                     "max_abs_dE_batched_vs_looped_eV": dE,
                     "status_batched": rb.status, "status_looped_worst": max(st_loop)}
    kw = dict(strain=S, B=w.B, nb=out["mixed"]["nb"], tol=1e-5, precision="mixed")
    t0 = time.perf_counter()
    rc = hkp.solve_sweep(V, w.h, w.nev, graph=True, stride=8, **kw)
    torch.cuda.synchronize()
    t_cont = time.perf_counter() - t0
    errs = {}
    for i in (0, 31, 63):
        ref, _, _ = _golden(f"sweep64_dqd_192x40x40_i{i}")
        errs[str(i)] = float(np.abs(res["mixed"].E[i].cpu().numpy() - ref).max())
    out.update({
        "speedup_batched_mixed_vs_looped_fp64": round(
            out["fp64"]["s_per_hamiltonian_looped"] / out["mixed"]["s_per_hamiltonian_batched_graph"], 3),
        "s_per_hamiltonian_continuation_mixed_graph": round(t_cont / 64, 5),
        "continuation": "every 8th member cold, the rest from the nearest one's psi",
        "max_abs_dE_continuation_vs_batched_eV": float((rc.E - res["mixed"].E).abs().max()),
        "status_continuation": rc.status,
        "max_abs_dE_batched_mixed_vs_oracle_eV": errs})
    return out


def adjoint_measure(torch, hkp, workload, reps=10):
    """Hellmann-Feynman backward of loss = sum of the lowest 8 eigenvalues in the 5
    gate voltages (192 x 40 x 40, B = 0): the warm backward (mean of `reps` calls,
    including the host-side check of equal weights within degenerate pairs), the
    library's gradient call alone (HIP events on the stream it runs on, mean of 20)
    against its HBM roofline, and the gradient's error against central finite
    differences (dV = 1e-4 V)."""
    w = workload("adjoint_dqd_192x40x40")
    Ld = torch.from_numpy(w.extra["L"]).cuda()
    Vbg = torch.from_numpy(w.V).cuda()
    S = torch.from_numpy(w.strain).cuda()
    nev, G = 8, Ld.shape[0]
    cfg = dict(h=w.h, nev=nev, strain=S, B=w.B, nb=16, tol=1e-10)
    Vg = torch.zeros(G, dtype=torch.float64, device="cuda", requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E = hkp.EigvalsFromPotential.apply(Vg, Ld, Vbg, cfg)
    loss = E.sum()
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    loss.backward(retain_graph=True)
    torch.cuda.synchronize()
    t_cold = time.perf_counter() - t0
    grad = Vg.grad.cpu().numpy().copy()
    t0 = time.perf_counter()
    for _ in range(reps):
        loss.backward(retain_graph=True)
    torch.cuda.synchronize()
    t_warm = (time.perf_counter() - t0) / reps
    # the library call alone, on the current stream (the one the binding passes)
    psi = hkp.solve(Vbg, w.h, nev, strain=S, B=w.B, nb=16, tol=1e-10).psi
    wts = torch.ones(nev, dtype=torch.float64, device="cuda")
    L2 = Ld.reshape(G, -1)
    hkp.hf_grad(psi, wts, L2)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        hkp.hf_grad(psi, wts, L2)
    e1.record()
    e1.synchronize()
    t_k = e0.elapsed_time(e1) * 1e-3 / 20
    N = int(np.prod(w.shape))
    alg = nev * N * 96 + G * N * 8   # psi read once, lever arms read once

    def esum(vg):
        V = Vbg + torch.tensordot(torch.as_tensor(vg, device="cuda"), Ld, dims=1)
        return float(hkp.solve(V, w.h, nev, strain=S, B=w.B, nb=16, tol=1e-10,
                               return_psi=False).E.sum())

    d = 1e-4
    fd = np.array([(esum(d * np.eye(G)[k]) - esum(-d * np.eye(G)[k])) / (2 * d)
                   for k in range(G)])
    return {"workload": "adjoint_dqd_192x40x40", "forward_s": round(t_fwd, 4),
            "backward_s_first": round(t_cold, 6), "backward_s_warm": round(t_warm, 6),
            "backward_reps": reps,
            "hf_grad_call_us": round(t_k * 1e6, 2),
            "host_side_s_per_backward": round(max(t_warm - t_k, 0.0), 6),
            "hf_roofline": {"bound": "hbm", "kernel": "hf_partial_kernel + hf_reduce_kernel",
                            "algorithmic_bytes": alg,
                            "achieved": round(alg / t_k / 1e9, 1), "peak": HBM_PEAK_GBPS,
                            "unit": "GB/s", "frac": round(alg / t_k / 1e9 / HBM_PEAK_GBPS, 4)},
            "grad_rel_err_vs_fd": float(np.abs(grad - fd).max() / np.abs(fd).max())}


# algorithmic bytes per node of one conjugate-gradient iteration of the Poisson
# solve: direction update + operator (read z, p, three link coefficients and the
# electrode mask, write p and L p) and the vector update (read D^-1, p, L p, phi,
# r; write phi, r, z)
CG_BYTES_PER_NODE = (8 + 8 + 24 + 1 + 8 + 8) + (5 * 8 + 3 * 8)
# one multigrid-preconditioned CG iteration, per node of the box: the operator (57, as
# above), the CG update fused into the finest restriction (read p, q, phi, r, D^-1,
# diag, three link weights = 72; write phi, the new r = 16; the coarse right-hand side
# 1), the finest correction (read r, D^-1, diag, three link weights = 48, the coarse
# correction 1; write z 8) and the coarser levels (the same pattern on 1/8 + 1/64 + ...
# of the nodes, about 15)
MG_PCG_BYTES_PER_NODE = 57 + (72 + 16 + 1) + (48 + 1 + 8) + 15


def sp_measure(torch, hkp, anneal_K=15.0):
    """Self-consistent Schroedinger-Poisson loop on the 256 x 48 x 48 double-dot fin
    inside a 272 x 64 x 88 Poisson box (1.53M nodes), two holes at 1.5 K, mixed
    precision eigensolves to 1e-7 eV, stopped at max |phi_out - phi_in| <= 1e-6 V:
    annealed from anneal_K (the main figures), then the direct loop at 1.5 K for
    comparison, both with the eigensolves' filter in product form (the loop's
    default), and the annealed loop with the three-term recurrence beside them;
    and the Poisson CG iteration rate against the HBM roofline (HIP
    events around a fixed number of iterations on the library's stream)."""
    from synth import sp_device
    d = sp_device("sp_dqd_256x48x48")
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda()
    eps, dirm, phif = t(d.eps_r), t(d.dirichlet), t(d.phi_fixed)
    kw = dict(strain=t(d.strain), B=d.B, nb=d.nb, tol=1e-7, precision="mixed", graph=True,
              tol_V=1e-6, cg_tol=1e-12, mixing=0.3, history=5)

    def loop(anneal_T):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = hkp.sp_solve(t(d.V_off), d.h, d.nev, d.pshape, d.offset, eps, dirm, phif,
                         d.n_holes, d.T, anneal_T=anneal_T, **kw)
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    r, wall = loop(anneal_K)
    direct, wall_direct = loop(0.0)
    kw["cheb_product"] = False   # the same loop with the eigensolves' filter as a recurrence
    rec, wall_rec = loop(anneal_K)
    kw.pop("cheb_product")
    st = r.stats
    NP = int(np.prod(d.pshape))
    return {"workload": "sp_dqd_256x48x48", "grid": list(d.shape), "poisson_box": list(d.pshape),
            "poisson_nodes": NP, "n_holes": d.n_holes, "T_K": d.T, "nev": d.nev, "nb": d.nb,
            "precision": "mixed", "stop": "max |phi_out - phi_in| <= 1e-6 V, eigen tol 1e-7 eV",
            "filter": "product form (the loop's default)",
            "anneal_K": anneal_K, "anneal_iterations": st["anneal_iters"],
            "status": r.status, "sp_iterations": st["iters"], "converged": st["converged"],
            "delta_V": st["delta_V"], "seconds": round(wall, 3),
            "s_per_sp_iteration": round(wall / max(st["iters"], 1), 4),
            "t_schroedinger_s": round(st["t_schroedinger"], 3),
            "t_poisson_s": round(st["t_poisson"], 3), "cg_iterations": st["cg_iters"],
            "eigensolver_iterations": st["schroedinger_iters"],
            "E0_eV": float(r.E[0]), "mu_eV": st["mu_eV"],
            "direct": {"sp_iterations": direct.stats["iters"],
                       "converged": direct.stats["converged"], "seconds": round(wall_direct, 3),
                       "max_abs_dE_vs_annealed_eV": float((direct.E - r.E).abs().max()),
                       "max_abs_dphi_vs_annealed_V": float((direct.phi - r.phi).abs().max())},
            "recurrence": {"sp_iterations": rec.stats["iters"], "converged": rec.stats["converged"],
                           "seconds": round(wall_rec, 3),
                           "t_schroedinger_s": round(rec.stats["t_schroedinger"], 3),
                           "max_abs_dE_vs_product_eV": float((rec.E - r.E).abs().max()),
                           "max_abs_dphi_vs_product_V": float((rec.phi - r.phi).abs().max())},
            "poisson_cg": poisson_measure(torch, hkp, d, r.density)}


def poisson_measure(torch, hkp, d=None, density=None, iters=1024):
    """Poisson CG on the 272 x 64 x 88 box, timed with HIP events on the library's
    stream: the multigrid-preconditioned solve to |r| <= 1e-12 |b| from zero (the
    library's default), and the Jacobi-preconditioned one both to the same tolerance
    and over a fixed iteration count (unreachable tolerance); per-iteration rates
    against the HBM roofline at MG_PCG_BYTES_PER_NODE and CG_BYTES_PER_NODE
    algorithmic bytes per node."""
    from synth import sp_device
    d = d or sp_device("sp_dqd_256x48x48")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    eps, dirm, phif = t(d.eps_r), t(d.dirichlet), t(d.phi_fixed)
    NP = int(np.prod(d.pshape))
    rho = torch.zeros(d.pshape, dtype=torch.float64, device="cuda")
    if density is None:   # two holes spread over the fin
        density = torch.full(d.shape, d.n_holes / (np.prod(d.shape) * d.h ** 3),
                             dtype=torch.float64, device="cuda")
    rho[d.offset[0]:d.offset[0] + d.shape[0], d.offset[1]:d.offset[1] + d.shape[1],
        d.offset[2]:d.offset[2] + d.shape[2]] = density
    def timed(**kw):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        _, it, rel, _ = hkp.poisson(eps, dirm, phif, rho, d.h, **kw)
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) * 1e-3, it, rel

    def rate(bpn, t_it):
        g = bpn * NP / t_it / 1e9
        return {"bytes_per_node": bpn, "achieved_gbps": round(g, 1), "peak_gbps": 8000.0,
                "frac": round(g / 8000.0, 4)}

    out = {"nodes": NP}
    prev = hkp.poisson_preconditioner("multigrid")
    try:
        timed(tol=1e-12)   # warm-up (graph recording)
        t, it, rel = timed(tol=1e-12)
        out["multigrid"] = {"s_to_1e-12": round(t, 5), "iterations": it, "relres": rel,
                            "us_per_iteration": round(t / it * 1e6, 2), **rate(MG_PCG_BYTES_PER_NODE, t / it)}
        hkp.poisson_preconditioner("jacobi")
        timed(tol=1e-30, max_iter=64)
        t, it, rel = timed(tol=1e-12)
        out["jacobi"] = {"s_to_1e-12": round(t, 5), "iterations": it, "relres": rel}
        t, it, _ = timed(tol=1e-30, max_iter=iters)
        out["jacobi"].update({"us_per_iteration": round(t / it * 1e6, 2),
                              "iterations_timed": it, **rate(CG_BYTES_PER_NODE, t / it)})
    finally:
        hkp.poisson_preconditioner(prev)
    out["speedup_to_solution"] = round(out["jacobi"]["s_to_1e-12"] / out["multigrid"]["s_to_1e-12"], 2)
    return out


def spin_free_measure(torch, hkp, workload):
    """Spin-free single-particle basis on the 256 x 48 x 48 double dot at B = 0
    (strain on): the 16 lowest orbitals of H_0 (three-component vectors) against
    the 32 lowest spinor states of the full Hamiltonian at B = 0 (the same number
    of states once spin is counted), both FP64 to residual 1e-8 eV, and the
    spin-orbit matrix of the 16 orbitals (32 x 32)."""
    w = workload(WORKLOAD)
    V = torch.from_numpy(w.V).cuda()
    S = torch.from_numpy(w.strain).cuda()
    kw = dict(strain=S, tol=1e-8, return_psi=False)
    for nb in (24, 40):   # stencil launch shapes for both block sizes (B = 0, strain)
        hkp.autotune(w.shape, w.h, nb, "fp64", with_field=False)
    hkp.solve(V, w.h, 16, nb=24, spin_free=True, **kw)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = hkp.solve(V, w.h, 16, nb=24, spin_free=True, strain=S, tol=1e-8)
    torch.cuda.synchronize()
    t_sf = time.perf_counter() - t0
    t0 = time.perf_counter()
    full = hkp.solve(V, w.h, 32, nb=40, **kw)
    torch.cuda.synchronize()
    t_full = time.perf_counter() - t0
    H = hkp.soi_matrix(r.psi, E=r.E)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        H = hkp.soi_matrix(r.psi, E=r.E)
    torch.cuda.synchronize()
    t_soi = (time.perf_counter() - t0) / 10
    ev = torch.linalg.eigvalsh(H).cpu().numpy()

    def stencil_rate(st):   # the library's event-timed FP64 stencil launches of one solve
        n, t, b = st["n_stencil64"], st["t_stencil64"], st["bytes_stencil64"]
        return {"launches": n, "avg_us": round(1e6 * t / max(n, 1), 1),
                "gbps": round(b / t / 1e9, 1) if t > 0 else None,
                "frac": round(b / t / 8e12, 4) if t > 0 else None}

    return {"workload": WORKLOAD + " at B = 0", "orbitals": 16,
            "stencil_fp64_orbital": stencil_rate(r.stats),
            "stencil_fp64_spinor": stencil_rate(full.stats),
            "s_spin_free_fp64": round(t_sf, 4), "iters_spin_free": r.stats["iters"],
            "s_full_32_states_fp64": round(t_full, 4), "iters_full": full.stats["iters"],
            "speedup": round(t_full / t_sf, 3), "s_soi_matrix_32x32": round(t_soi, 6),
            "status": [r.status, full.status],
            "lowest_single_particle_eV": [float(v) for v in ev[:4]],
            "lowest_full_eV": [float(v) for v in full.E[:4].cpu().numpy()]}


def _hole_free_device(torch, hkp):
    """The 256 x 48 x 48 double-dot fin in its 272 x 64 x 88 box: the potential of
    the gates alone (one Poisson solve), its strain, permittivity and electrodes."""
    from synth import sp_device
    d = sp_device("sp_dqd_256x48x48")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    eps, dirm = t(d.eps_r), t(d.dirichlet)
    phi0, _, _, _ = hkp.poisson(eps, dirm, t(d.phi_fixed), None, d.h, tol=1e-12)
    ox, oy, oz = d.offset
    V = t(d.V_off) + phi0[ox:ox + d.shape[0], oy:oy + d.shape[1], oz:oz + d.shape[2]]
    return d, V, t(d.strain), eps, dirm


def ci_measure(torch, hkp, dev=None):
    """Two-hole configuration interaction on the 256 x 48 x 48 double-dot fin in its
    272 x 64 x 88 box (hole-free potential, B = 0, strain): 4 spin-free orbitals,
    28 determinants, the 10 pair potentials (16 nonzero real right-hand sides) from
    one batched CG solve to |r| <= 1e-11 |b|."""
    d, V, S, eps, dirm = dev if dev is not None else _hole_free_device(torch, hkp)
    hkp.solve(V, d.h, 4, strain=S, nb=12, tol=1e-9, spin_free=True)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = hkp.solve(V, d.h, 4, strain=S, nb=12, tol=1e-9, spin_free=True)
    torch.cuda.synchronize()
    t_orb = time.perf_counter() - t0
    t0 = time.perf_counter()
    ci = hkp.ci_solve(r.psi, r.E, d.h, d.pshape, d.offset, eps, dirm, cg_tol=1e-11)
    torch.cuda.synchronize()
    t_ci = time.perf_counter() - t0
    st = ci.stats
    per = st["t_poisson"] / max(1, st["cg_iters"] * st["poisson_solves"])   # per nonzero rhs
    nodes = int(np.prod(d.pshape))
    cg_rate = MG_PCG_BYTES_PER_NODE * nodes / per   # algorithmic bytes per iteration and rhs
    return {"workload": "sp_dqd_256x48x48, hole-free potential, B = 0", "orbitals": 4,
            "determinants": st["determinants"], "s_orbitals": round(t_orb, 4),
            "s_ci": round(t_ci, 4), "poisson_right_hand_sides": st["poisson_solves"],
            "cg_iterations": st["cg_iters"], "s_poisson_batched": round(st["t_poisson"], 4),
            "us_per_cg_iteration_per_rhs": round(per * 1e6, 2),
            "cg_roofline": {"bound": "hbm", "bytes_per_node": MG_PCG_BYTES_PER_NODE,
                            "achieved_gbps": round(cg_rate / 1e9, 1), "peak_gbps": 8000.0,
                            "frac": round(cg_rate / 8e12, 4)},
            "J_eV": ci.J,
            "lowest_two_hole_eV": [float(v) for v in ci.E[:4].cpu().numpy()],
            "status": ci.status}


def qubit_measure(torch, hkp, J=None, dev=None):
    """g-matrices of the lowest two Kramers doublets (FP64 solve to 1e-10 at B = 0) on
    the same hole-free potential as the CI, and the effective two-spin model over a
    1-degree map of field orientations at |B| = 50 mT, with the CI's J.  The spin-orbit
    axis and length come from measurements the paper cites and does not print; n_so = z
    and lambda_so = 50 nm stand in for them."""
    d, V, S, eps, dirm = dev if dev is not None else _hole_free_device(torch, hkp)
    if J is None:
        r = hkp.solve(V, d.h, 4, strain=S, nb=12, tol=1e-9, spin_free=True)
        J = hkp.ci_solve(r.psi, r.E, d.h, d.pshape, d.offset, eps, dirm, cg_tol=1e-11).J
    r = hkp.solve(V, d.h, 4, strain=S, tol=1e-10)
    hkp.g_matrices(r.psi, V, d.h, strain=S)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gm = hkp.g_matrices(r.psi, V, d.h, strain=S)
    t_g = time.perf_counter() - t0
    th = np.radians(np.arange(0, 181))
    ph = np.radians(np.arange(0, 361))
    T, P = np.meshgrid(th, ph, indexing="ij")
    Bd = 0.05 * np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1)
    Bt = torch.from_numpy(Bd.reshape(-1, 3)).cuda()
    n_so, lam = (0.0, 0.0, 1.0), 50.0
    hkp.two_spin_model(gm, J, Bt, n_so, lam)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = hkp.two_spin_model(gm, J, Bt, n_so, lam)
    torch.cuda.synchronize()
    t_m = time.perf_counter() - t0
    jp = out["J_perp"].cpu().numpy().reshape(T.shape)
    jl = out["J_par"].cpu().numpy().reshape(T.shape)
    dz = out["dEz"].cpu().numpy().reshape(T.shape)
    at = lambda k: [int(v) for v in np.unravel_index(k, T.shape)]
    # algorithmic bytes of one g-matrix call, in spinor blocks of 6 N complex doubles:
    # 4 in + 4 out (layout), 4 + 12 (position weights), 16 + 16 (stencil), 4 + 12 (Zeeman),
    # 44 (the Gram product reads each vector once)
    blk = 6 * int(np.prod(d.shape)) * 16
    g_bytes = 116 * blk
    return {"workload": "sp_dqd_256x48x48, hole-free potential; |B| = 50 mT, 181 x 361 "
                        "orientations", "s_g_matrices": round(t_g, 5),
            "g_matrices_gbps_algorithmic": round(g_bytes / t_g / 1e9, 1),
            "s_two_spin_model": round(t_m, 5), "orientations": int(Bt.shape[0]),
            "g_left": np.round(gm.g_sym[2], 4).tolist(), "g_right": np.round(gm.g_sym[3], 4).tolist(),
            "delta_eV": gm.delta, "t_eV": gm.t, "d_nm": round(gm.d, 3), "J_eV": J,
            "U_minus_eps_eV": 2 * gm.t ** 2 / J if J else None,
            "max_J_perp": [float(jp.max()), at(jp.argmax())],
            "min_J_perp": [float(jp.min()), at(jp.argmin())],
            "J_par_at_min_J_perp": float(jl.flat[jp.argmin()]),
            "max_dEz_over_J_perp": float((dz / np.maximum(jp, 1e-300)).max()),
            "kramers_defect": float(np.abs(gm.kramers[:2]).max())}


def cpu_baseline(w, seconds, oracle_matvecs, oracle_solve_s, workload):
    """The CPU oracle on this host: its H.X (scipy CSR matvec on the assembled
    Hamiltonian) on a slab of the bench workload, in the metric's unit; a solve
    time for the full workload extrapolated from it (ARPACK's operator-application
    count of the oracle's reference run times the measured single-vector matvec
    time of the whole grid; ARPACK's own orthogonalisation is not included, so
    this is a lower bound); and one complete oracle solve, the dense LAPACK
    diagonalisation of the 10 x 8 x 8 harmonic workload (3840 unknowns)."""
    from oracle import SI_MATERIAL, Grid, hamiltonian_ls, lowest_dense
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max((d.get("num_threads", 1) for d in threadpool_info()
                            if d.get("user_api") == "blas"), default=None)
    except Exception:   # threadpoolctl absent: thread count unknown
        blas_threads = None
    nxs = 32   # slab: the first 32 x-planes of the 256 x 48 x 48 grid
    g = Grid(nxs, w.ny, w.nz, w.h)
    t0 = time.perf_counter()
    H = hamiltonian_ls(g, SI_MATERIAL, w.V[:nxs].ravel(), w.strain[:nxs].reshape(-1, 6), w.B)
    t_asm = time.perf_counter() - t0
    nvec = 8
    rng = np.random.default_rng(0)
    X = rng.standard_normal((H.shape[0], nvec)) + 1j * rng.standard_normal((H.shape[0], nvec))
    reps = 0
    t0 = time.perf_counter()
    while True:
        _ = H @ X
        reps += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    bytes_ = reps * nvec * g.npts * 6 * 16 * 2.0   # read X, write Y (complex FP64)
    # one vector at a time, as ARPACK applies the operator
    x = X[:, 0].copy()
    k1 = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < min(3.0, seconds / 4):
        _ = H @ x
        k1 += 1
    t_mv_full = (time.perf_counter() - t0) / k1 * (w.nx / nxs)
    # the dense oracle solve of the small harmonic workload
    c1 = workload("harmonic_10x8x8")
    H1 = hamiltonian_ls(Grid(c1.nx, c1.ny, c1.nz, c1.h), SI_MATERIAL, c1.V)
    t0 = time.perf_counter()
    lowest_dense(H1, c1.nev)
    t_c1 = time.perf_counter() - t0
    return dict(value=bytes_ / dt / 1e9, unit="GB/s", cores=1, kind="oracle",
                sample=(f"oracle CSR H.X (scipy, single-threaded matvec) on the first {nxs} x-planes "
                        f"of the {WORKLOAD} workload ({g.npts} points, {H.nnz} non-zeros), "
                        f"{nvec} complex vectors x {reps} repetitions in {dt:.1f} s; "
                        f"assembly {t_asm:.1f} s not included; host cpu_count {os.cpu_count()}"),
                s_per_solve_extrapolated=(round(oracle_matvecs * t_mv_full, 1)
                                          if oracle_matvecs else None),
                extrapolation=(f"{oracle_matvecs} ARPACK operator applications (the oracle's "
                               f"reference solve of {WORKLOAD} to tol 1e-11) x {t_mv_full:.4f} s "
                               f"per single-vector CSR matvec of the whole grid (slab time x "
                               f"{w.nx // nxs}); orthogonalisation not counted: a lower bound"
                               if oracle_matvecs else "matvec count not recorded"),
                reference_solve_s_elsewhere=oracle_solve_s,
                reference_solve_note=("wall time of that reference ARPACK solve where the golden "
                                      "file was made (8-core build container), not this host"),
                c1_dense_eigh_s=round(t_c1, 3),
                c1_workload="harmonic_10x8x8 (3840 unknowns), LAPACK evr, lowest 8",
                c1_blas_threads=blas_threads)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also copy a 1 GiB buffer (reference for HBM byte counters)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the sweep, adjoint and copy-bandwidth measurements")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--stencil", metavar="TY,VGROUP,DMA",
                    help="use this stencil launch shape instead of autotuning (profiled runs)")
    ap.add_argument("--nb", type=int, default=0,
                    help="use this block size instead of autotuning it (profiled runs)")
    ap.add_argument("--sp-only", action="store_true",
                    help="run only the self-consistent loop measurement (profiled runs); "
                         "prints its JSON object")
    ap.add_argument("--poisson-only", action="store_true",
                    help="run only the Poisson CG rate measurement (profiled runs)")
    ap.add_argument("--spin-free-only", action="store_true",
                    help="run only the spin-free basis measurement (profiled runs)")
    ap.add_argument("--ci-only", action="store_true",
                    help="run only the configuration-interaction measurement (profiled runs)")
    ap.add_argument("--qubit-only", action="store_true",
                    help="run only the g-matrix / two-spin-model measurement (profiled runs)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the Hellmann-Feynman backward measurement (profiled runs)")
    ap.add_argument("--fp64-solve-only", action="store_true",
                    help="one FP64 solve of the benchmark workload (residual 1e-5 eV) and its "
                         "FP64 stencil statistics (profiled runs of the FP64 stencil)")
    ap.add_argument("--bench-log", default=None,
                    help="with --traffic-from: stdout of the profiled benchmark run")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"],
                    help="with --traffic-from: which stencil's dispatches to summarise")
    args = ap.parse_args()
    if args.traffic_from:
        if not args.stencil or not args.nb:
            raise SystemExit("--traffic-from needs --stencil TY,VGROUP,DMA and --nb NB "
                             "(the profiled launch shape and block size)")
        traffic_from(*args.traffic_from, args.stencil, args.nb, args.precision, args.bench_log)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    if args.stencil:
        os.environ["HKP_STENCIL"] = args.stencil
    import torch
    import paper_2607_08447_amd as hkp
    from synth import workload

    if args.copy_calibration:
        src_buf = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        dst_buf = torch.empty_like(src_buf)
        dst_buf.copy_(src_buf)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")
        del src_buf, dst_buf

    if args.sp_only:
        print(json.dumps(sp_measure(torch, hkp)), flush=True)
        return
    if args.poisson_only:
        print(json.dumps(poisson_measure(torch, hkp)), flush=True)
        return
    if args.spin_free_only:
        print(json.dumps(spin_free_measure(torch, hkp, workload)), flush=True)
        return
    if args.ci_only:
        print(json.dumps(ci_measure(torch, hkp)), flush=True)
        return
    if args.qubit_only:
        print(json.dumps(qubit_measure(torch, hkp)), flush=True)
        return
    if args.adjoint_only:
        print(json.dumps(adjoint_measure(torch, hkp, workload)), flush=True)
        return
    if args.fp64_solve_only:
        w = workload(WORKLOAD)
        r = hkp.solve(torch.from_numpy(w.V).cuda(), w.h, 32, strain=torch.from_numpy(w.strain).cuda(),
                      B=w.B, nb=args.nb or 40, tol=1e-5, precision="fp64", return_psi=False)
        torch.cuda.synchronize()
        st = r.stats
        print(json.dumps({"status": r.status, "iters": st["iters"],
                          "n_stencil64": st["n_stencil64"],
                          "algorithmic_bytes_per_launch": st["bytes_stencil64"] / max(st["n_stencil64"], 1),
                          "avg_launch_us": 1e6 * st["t_stencil64"] / max(st["n_stencil64"], 1)}),
              flush=True)
        return

    w = workload(WORKLOAD)
    nev, tol = 32, 1e-5
    V = torch.from_numpy(w.V).cuda()
    S = torch.from_numpy(w.strain).cuda()
    log(f"workload {WORKLOAD} {w.shape} h={w.h} nev={nev}")
    # block size per precision: measured (one solve per candidate) unless forced
    nbs, nb_tuning = {}, {}
    for prec in ("mixed", "fp64"):
        if args.nb:
            nbs[prec] = args.nb
        else:
            t = hkp.autotune_block(V, w.h, nev, strain=S, B=w.B, candidates=[40, 48, 56],
                                   tol=tol, precision=prec)
            nbs[prec], nb_tuning[prec] = t["nb"], t["seconds"]
    log(f"block size {nbs} {nb_tuning}")
    if args.stencil:
        ty, vg, dma = (int(v) for v in args.stencil.split(","))
        tune64 = tune32 = {"tile_y": ty, "vgroup": vg, "dma": dma, "forced": True}
    else:
        tune64 = hkp.autotune(w.shape, w.h, nbs["fp64"], "fp64")
        tune32 = hkp.autotune(w.shape, w.h, nbs["mixed"], "mixed")
    log(f"stencil launch shape: fp64 {tune64} fp32 {tune32}")
    ws = torch.empty(max(hkp.workspace_bytes(w.shape, w.h, nev, nb=nbs["mixed"], precision="mixed"),
                         hkp.workspace_bytes(w.shape, w.h, nev, nb=nbs["fp64"], precision="fp64")),
                     dtype=torch.uint8, device="cuda")

    def solve(prec, t, product=False):
        # eigenvectors returned (|J m_j> basis, symmetric gauge, ABI layout): the
        # output step is part of every timed solve
        return hkp.solve(V, w.h, nev, strain=S, B=w.B, nb=nbs[prec], tol=t, precision=prec,
                         workspace=ws, return_psi=True, cheb_product=product)

    t0 = time.perf_counter()
    ref = solve("fp64", 1e-8)
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0
    E_ref = ref.E.cpu().numpy()
    log(f"reference FP64 solve (tol 1e-8): {t_ref:.3f} s, status {ref.status}")

    for _ in range(args.warmup):
        solve("mixed", tol)
    torch.cuda.synchronize()
    stats = []
    errs = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        r = solve("mixed", tol)
        stats.append(r.stats)
        errs.append(r.E)
        log(f"step {k}: status {r.status}, iters {r.stats['iters']}")
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    err_mixed = max(float(np.abs(e.cpu().numpy() - E_ref).max()) for e in errs)
    E_oracle, oracle_matvecs, oracle_solve_s = _golden(WORKLOAD)
    # per state, the largest error over the timed steps
    per_mixed = np.max([np.abs(e.cpu().numpy() - E_oracle) for e in errs], axis=0)
    per_ref = np.abs(E_ref - E_oracle)

    t0 = time.perf_counter()
    r64 = solve("fp64", tol)
    torch.cuda.synchronize()
    t_fp64 = time.perf_counter() - t0
    err_fp64 = float(np.abs(r64.E.cpu().numpy() - E_ref).max())
    per_fp64 = np.abs(r64.E.cpu().numpy() - E_oracle)
    log(f"FP64 solve (tol {tol}): {t_fp64:.3f} s, max |dE| {err_fp64:.2e}")

    # the same solves with the filter in product form (the same polynomial over
    # its roots: one block read and one written per step instead of two read)
    log("product-form filter ...")
    solve("mixed", tol, product=True)
    torch.cuda.synchronize()
    pstats, perrs, pstatus = [], [], []
    t0 = time.perf_counter()
    for k in range(args.steps):
        r = solve("mixed", tol, product=True)
        pstats.append(r.stats)
        perrs.append(r.E)
        pstatus.append(int(r.status))
    torch.cuda.synchronize()
    t_prod = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    r64p = solve("fp64", tol, product=True)
    torch.cuda.synchronize()
    t_prod64 = time.perf_counter() - t0
    pn32 = sum(s["n_stencil32"] for s in pstats)
    pb32 = sum(s["bytes_stencil32"] for s in pstats) / max(pn32, 1)
    pt32 = sum(s["t_stencil32"] for s in pstats) / max(pn32, 1)
    product_form = {
        "s_per_solve_mixed": round(t_prod, 4),
        "s_per_solve_fp64": round(t_prod64, 4),
        "hx_gbps": round(sum(s["hx_bytes"] for s in pstats) / (t_prod * args.steps) / 1e9, 1),
        "iters_mixed": pstats[-1]["iters"], "iters_fp64": r64p.stats["iters"],
        "max_err_mixed_vs_oracle_eV": float(max(np.abs(e.cpu().numpy() - E_oracle).max()
                                                for e in perrs)),
        "max_err_fp64_vs_oracle_eV": float(np.abs(r64p.E.cpu().numpy() - E_oracle).max()),
        "stencil_fp32": {"launches": pn32, "algorithmic_bytes_per_launch": pb32,
                         "avg_launch_us": round(pt32 * 1e6, 1),
                         "gbps": round(pb32 / max(pt32, 1e-12) / 1e9, 1),
                         "frac": round(pb32 / max(pt32, 1e-12) / 1e9 / HBM_PEAK_GBPS, 4)},
        "status_mixed": max(pstatus), "status_fp64": int(r64p.status),
    }
    log(f"product form {product_form}")

    hx_bytes = sum(s["hx_bytes"] for s in stats)
    n32 = sum(s["n_stencil32"] for s in stats)
    t32 = sum(s["t_stencil32"] for s in stats)
    b32 = sum(s["bytes_stencil32"] for s in stats)
    bytes_per_launch = b32 / max(n32, 1)
    avg_launch = t32 / max(n32, 1)
    achieved = bytes_per_launch / avg_launch / 1e9
    traffic = _traffic_for(_src_hash(), _shape_key(tune32, nbs["mixed"]), bytes_per_launch)
    extra = {}
    if not args.no_extra:
        log("copy bandwidth ...")
        extra["copy_gbps"] = round(copy_bandwidth(torch), 1)
        extra["triad_gbps"] = round(triad_bandwidth(torch), 1)
        log("sweep: 64 Hamiltonians batched vs looped ...")
        extra["sweep"] = sweep_measure(torch, hkp, workload)
        log(f"sweep {extra['sweep']}")
        log("adjoint ...")
        extra["adjoint"] = adjoint_measure(torch, hkp, workload)
        log(f"adjoint {extra['adjoint']}")
        log("spin-free basis ...")
        extra["spin_free"] = spin_free_measure(torch, hkp, workload)
        log(f"spin-free {extra['spin_free']}")
        log("configuration interaction ...")
        dev = _hole_free_device(torch, hkp)
        extra["ci"] = ci_measure(torch, hkp, dev)
        log(f"ci {extra['ci']}")
        log("g-matrices and the two-spin model ...")
        extra["qubit"] = qubit_measure(torch, hkp, extra["ci"]["J_eV"], dev)
        log(f"qubit {extra['qubit']}")
        log("self-consistent Schroedinger-Poisson loop ...")
        extra["sp"] = sp_measure(torch, hkp)
        log(f"sp {extra['sp']}")

    out = {
        "metric": METRIC,
        "value": round(hx_bytes / t_steps / 1e9, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_steps / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 filter / c128 orth+RR+residual",
        "data": "synthetic (seeded DQD fin potential, strain, B field)",
        "config": {"workload": WORKLOAD, "grid": list(w.shape), "h_nm": w.h, "nev": nev,
                   "nb": nbs["mixed"], "nb_fp64": nbs["fp64"],
                   "nb_tuning_s": nb_tuning or "forced",
                   "precision": "mixed", "stop": "per-state residual <= 1e-5 eV",
                   "B_T": list(w.B), "strain": "ezz -0.3% + smooth perturbation"},
        "s_per_solve_mixed": round(t_steps / args.steps, 4),
        "s_per_solve_fp64": round(t_fp64, 4),
        "s_per_solve_fp64_tol1e-8": round(t_ref, 4),
        "speedup_mixed_vs_fp64": round(t_fp64 / (t_steps / args.steps), 3),
        "oracle": ("tests/golden/dqd_256x48x48.txt: the oracle's lowest 32 eigenvalues "
                   "(ARPACK on the assembled Hamiltonian)"),
        "err_per_state_mixed_eV": [float(v) for v in per_mixed],
        "err_per_state_fp64_eV": [float(v) for v in per_fp64],
        "err_per_state_fp64_tol1e-8_eV": [float(v) for v in per_ref],
        "max_err_mixed_vs_oracle_eV": float(per_mixed.max()),
        "max_err_fp64_vs_oracle_eV": float(per_fp64.max()),
        "max_err_fp64_tol1e-8_vs_oracle_eV": float(per_ref.max()),
        "within_1ueV": bool(per_mixed.max() <= 1e-6),
        "max_err_mixed_vs_fp64_ref_eV": err_mixed,
        "max_err_fp64_vs_fp64_ref_eV": err_fp64,
        "iters_mixed": stats[-1]["iters"],
        "iters_fp64": r64.stats["iters"],
        "roofline": {
            "bound": "hbm", "kernel": "stencil_kernel<float> (FP32 Chebyshev filter step)",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "avg_launch_us": round(avg_launch * 1e6, 1),
            "launches": n32,
            "frac_of_copy": (round(achieved / extra["copy_gbps"], 4)
                             if "copy_gbps" in extra else None),
            "frac_of_triad": (round(achieved / extra["triad_gbps"], 4)
                              if "triad_gbps" in extra else None),
        },
        "stencil_launch": {"fp32": tune32, "fp64": tune64},
        "filter": "three-term recurrence (Y_k+1 = alpha (H - c) Y_k + beta Y_k-1)",
        "product_form": product_form,
        "fp64_stencil_gbps": round(r64.stats["bytes_stencil64"] /
                                   max(r64.stats["t_stencil64"], 1e-12) / 1e9, 1),
    }
    out.update(extra)
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds, oracle_matvecs, oracle_solve_s,
                                           workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
