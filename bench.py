"""Benchmark: permeability solves per second on one MI355X.

Workload (default): FP64 solve on a 256^3 periodic box of overlapping solid
spheres of radius 3 voxels packed to porosity 0.2 (seed 0; high
surface-to-volume ratio), unit body force along x, outer CG on the pressure
Schur complement with the SIMPLE preconditioner to a relative residual of
1e-8, inner tolerances 1e-12.  One step is one full solve from p = 0 on a
context whose geometry is resident in HBM (setup, which reads a host mask,
runs once before timing and is reported separately), followed by the
permeability read-back.  Beside it: the same solve in mixed precision, one
mixed-precision solve of the 512^3 Gaussian-random-field geometry, and a short
seeded stream of mixed-precision requests (box sides 32..128) through the
request server with its throughput and p50/p99 latency (`--serve-only
--requests 2000` runs the full serving workload alone).

The CPU baseline times the oracle's own inner iterations on the same
geometry on the host cores and scales them with the oracle's own Jacobi inner
iteration counts for this geometry, which `--oracle-counts` measures (a CPU
run of the oracle's first solves, minutes long) and stores under profiles/.

Prints one JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SERVE_SLOTS = 4              # the box's hardware queues (GPU_MAX_HW_QUEUES default)
SERVE_BUDGET = 8 << 30          # HBM budget of the request server (bytes)

# name: (description, side, generator)
WORKLOADS = {
    "spheres128": ("128^3 periodic overlapping spheres r=6 porosity 0.5 seed 0", 128,
                   lambda: __import__("synth").spheres(128, 6.0, 0.5, 0)),
    "tight256": ("256^3 periodic overlapping spheres r=3 porosity 0.2 seed 0", 256,
                 lambda: __import__("synth").spheres(256, 3.0, 0.2, 0)),
    "grf512": ("512^3 Gaussian random field corr length 8 porosity 0.15 seed 0", 512,
               lambda: __import__("synth").grf(512, 8.0, 0.15, 0)),
}


# `--study precond`: SIMPLE against Uzawa over surface-to-volume ratios at 128^3
# (the paper's Sec. 4.1.2 / 4.2.2 comparison).  Plane channels parallel to the
# force carry no pressure: there g = B A^-1 f is only the inner solve's error,
# so their outer counts measure iterations on that noise, not the preconditioner.
PRECOND_STUDY = [
    ("spheres r=10 porosity 0.7 seed 0", lambda: __import__("synth").spheres(128, 10.0, 0.7, 0)),
    ("spheres r=6 porosity 0.5 seed 0", lambda: __import__("synth").spheres(128, 6.0, 0.5, 0)),
    ("spheres r=4 porosity 0.4 seed 0", lambda: __import__("synth").spheres(128, 4.0, 0.4, 0)),
    ("spheres r=3 porosity 0.3 seed 0", lambda: __import__("synth").spheres(128, 3.0, 0.3, 0)),
    ("spheres r=3 porosity 0.2 seed 0", lambda: __import__("synth").spheres(128, 3.0, 0.2, 0)),
    ("slit stack, walls 2, widths 4 8 12 16 24 32, walls normal to y",
     lambda: __import__("synth").slits(128, [4, 8, 12, 16, 24, 32], 2, 1)),
]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stream_copy_gbps(torch, nbytes=1 << 30, reps=5):
    """Device-to-device copy rate (bytes read + bytes written per second), the
    practical streaming ceiling beside the published HBM peak; timed with events
    on the current stream after one untimed copy."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def precond_study(P, cases=None):
    """One JSON line per geometry: outer iterations, inner iterations and solve
    time of the FP64 solve (tol 1e-8) with each preconditioner."""
    import torch
    for desc, gen in (cases or PRECOND_STUDY):
        mask = gen()
        with P.Stokes(mask, (1.0, 0.0, 0.0)) as s:
            s.set_option("progress", 250)              # Uzawa may take thousands of outer iterations
            info = s.info()
            row = {"study": "precond", "geometry": desc, "N": info["N"],
                   "porosity": info["nfluid_in"] / info["N"] ** 3,
                   "stv_ratio": info["nsurf"] / max(1, info["nfluid_in"])}
            for name, pc in (("simple", P.STOKES_SIMPLE), ("uzawa", P.STOKES_UZAWA)):
                s.solve(pc, 1e-8)                      # graphs captured, caches warm
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rep = s.solve(pc, 1e-8)
                dt = time.perf_counter() - t0
                row[name] = {"outer_iters": rep["outer_iters"], "inner_A_iters": rep["inner_A_iters"],
                             "inner_S_iters": rep["inner_S_iters"], "seconds": dt, "k_hat": rep["k_hat"],
                             "status": rep["status"]}
                log(f"[study] {desc}: {name} outer={rep['outer_iters']} {dt:.3f} s k={rep['k_hat']:.10e}")
            ks, ku = row["simple"]["k_hat"], row["uzawa"]["k_hat"]
            row["k_rel_diff"] = abs(ks - ku) / abs(ks) if ks else 0.0
        print(json.dumps(row), flush=True)


def slit_study(P, torch, N=128, widths=(4, 6, 8, 12, 16, 24, 32), seeds=(0, 1, 2)):
    """The 128^3 slit stacks (walls 2 voxels thick, normal to y, channel width W):
    (i) force along the channels (g = 0: no outer step, plane Poiseuille flux),
    (ii) oblique force (1, 0.5, 0) (the flux of (i), pressure steps of f_y),
    (iii) random consistent right-hand sides g = B xi (xi seeded, standard
    normal on the faces) for the outer counts against the surface-to-volume
    ratio; FP64, tol 1e-8, both preconditioners.  One JSON line per width."""
    import numpy as np

    from synth import random_face_field, slits
    from synth.geometry import channel_widths
    for W in widths:
        m = slits(N, W, 2, 1)
        ws = channel_widths(N, W)
        kx = sum(w * (w * w + 2) / 12.0 for w in ws) / N
        row = {"study": "slits", "N": N, "W": W, "channels": len(ws), "kvox_closed_form": kx}
        with P.Stokes(m, (1.0, 0.0, 0.0)) as s:
            info = s.info()
            row["stv_ratio"] = info["nsurf"] / info["nfluid_in"]
            for pc in ("simple", "uzawa"):
                rep = s.solve(pc, 1e-8)
                row[f"i_{pc}"] = {"outer": rep["outer_iters"], "kvox_rel_err": abs(rep["k_vox"] - kx) / kx,
                                  "zero_rhs": bool(rep["flags"] & P.STOKES_FLAG_ZERO_RHS)}
            for q in seeds:
                xi = torch.tensor(random_face_field(N, q).reshape(-1), dtype=torch.float64, device="cuda")
                g = torch.empty(N ** 3, dtype=torch.float64, device="cuda")
                s.apply_device(P.STOKES_OP_B, xi, g)
                gh = g.cpu().numpy()
                for pc in ("simple", "uzawa"):
                    t0 = time.perf_counter()
                    rep = s.solve_rhs(gh, pc, 1e-8)
                    row.setdefault(f"iii_{pc}_outer", []).append(rep["outer_iters"])
                    row.setdefault(f"iii_{pc}_seconds", []).append(time.perf_counter() - t0)
        with P.Stokes(m, (1.0, 0.5, 0.0)) as s:
            for pc in ("simple", "uzawa"):
                rep = s.solve(pc, 1e-8)
                row[f"ii_{pc}"] = {"outer": rep["outer_iters"],
                                   "kvox_x_rel_err": abs(rep["mean_u"][0] - kx) / kx,
                                   "mean_u_y": rep["mean_u"][1]}
        log(f"[slits] W={W} stv={row['stv_ratio']:.3f} (iii) outer simple {row['iii_simple_outer']} "
            f"uzawa {row['iii_uzawa_outer']}")
        print(json.dumps(row), flush=True)


def batch_study(P, torch, members=(1, 4, 8, 16, 32), sides=(32, 48, 64)):
    """Mixed-precision SIMPLE solves of small boxes (spheres r=3, porosity 0.45):
    one batched context of B members against B contexts of one member solved
    one after another, time per request; one JSON line per size."""
    from synth import spheres
    for N in sides:
        row = {"study": "batch", "N": N, "workload": f"{N}^3 spheres r=3 porosity 0.45, mixed SIMPLE, tol 1e-8"}
        for B in members:
            if B * N ** 3 > (1 << 21) and B > 1:
                continue
            masks = [spheres(N, 3.0, 0.45, 7000 + q) for q in range(B)]
            with P.StokesBatch(masks) as b:
                b.solve("simple", 1e-8)                  # graphs captured, caches warm
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                reps = b.solve("simple", 1e-8)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
            row[f"batch_{B}_ms_per_request"] = dt / B * 1e3
            row[f"batch_{B}_outer_mean"] = sum(r["outer_iters"] for r in reps) / B
            log(f"[batch study] N={N} B={B}: {dt * 1e3:.1f} ms, {dt / B * 1e3:.2f} ms per request")
        print(json.dumps(row), flush=True)


def measured_traffic(kernel, N):
    """HBM bytes per launch of `kernel` from the committed hardware-counter summary,
    or None when that summary was taken at another size or on other kernel code
    (a hash of the kernel sources)."""
    import hashlib
    import re
    tables = {128: "traffic_128_spheres_inner_cg.md", 256: "traffic_256_tight_spheres.md"}
    if N not in tables:
        return None
    path = os.path.join(ROOT, "profiles", tables[N])
    srcs = [os.path.join(ROOT, "paper_2307_05266_amd", "csrc", f) for f in ("kernels.h", "mg.h")]
    try:
        m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
        table = json.loads(m.group(1))
        h = hashlib.sha256(b"".join(open(f, "rb").read() for f in srcs)).hexdigest()[:16]
    except (OSError, AttributeError, ValueError):
        return None
    if table.get("kernels_sha256_16") != h or table.get("N") != N:
        return None
    entry = table["per_launch"].get(kernel)
    return entry["traffic_bytes"] if entry else None


def _sha16(data: bytes) -> str:
    import hashlib
    return hashlib.sha256(data).hexdigest()[:16]


def oracle_counts_path(workload):
    return os.path.join(ROOT, "profiles", f"oracle_inner_counts_{workload}.md")


def read_json_block(path):
    """The JSON code block of a committed summary under profiles/."""
    import re
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        raise ValueError(f"no JSON block in {path}")
    return json.loads(m.group(1))


def oracle_source_hash():
    return _sha16(open(os.path.join(ROOT, "oracle", "stokes_oracle.c"), "rb").read())


def measure_oracle_counts(workload, outer=2):
    """CPU only: the oracle's own Jacobi-PCG inner iteration counts on a workload
    (its first inner solves: u0 = A^-1 f and the SIMPLE solve of g, then the
    first `outer` outer iterations), written to profiles/ for the CPU baseline."""
    import numpy as np
    import oracle
    desc, N, gen = WORKLOADS[workload]
    mask = gen()
    log(f"[oracle-counts] {desc}: assembling")
    t0 = time.perf_counter()
    o = oracle.Oracle(mask, (1.0, 0.0, 0.0))
    t_setup = time.perf_counter() - t0
    log(f"[oracle-counts] assembled in {t_setup:.1f} s: {o.nf} face and {o.nc} cell unknowns; solving "
        f"with max_outer={outer} on {oracle.threads()} threads")
    t0 = time.perf_counter()
    r = o.solve(oracle.SIMPLE, tol=1e-8, eps_A=1e-12, eps_S=1e-12, max_outer=outer)
    dt = time.perf_counter() - t0
    h = r["hist"]
    per_outer_A = [int(v) for v in h[:, 3]]
    per_outer_S = [int(v) for v in h[:, 4]]
    rec = {
        "workload": workload, "description": desc, "N": N,
        "mask_sha256_16": _sha16(np.ascontiguousarray(mask).tobytes()),
        "oracle_c_sha256_16": oracle_source_hash(),
        "precond": "simple", "eps_A": 1e-12, "eps_S": 1e-12,
        "start_A": int(r["inner_A"] - sum(per_outer_A)), "start_S": int(r["inner_S"] - sum(per_outer_S)),
        "per_outer_A": per_outer_A, "per_outer_S": per_outer_S,
        "outer_done": int(r["outer_iters"]), "seconds": dt, "threads": oracle.threads(),
        "command": f"python bench.py --oracle-counts --workload {workload}",
    }
    with open(oracle_counts_path(workload), "w") as f:
        f.write(f"# The oracle's own inner iteration counts on the {desc} workload\n\n"
                f"Command (repository root, CPU only): `{rec['command']}`\n\n"
                "The CPU oracle (FP64, CSR over the active unknowns, Jacobi-PCG inner solves to 1e-12) runs its\n"
                f"SIMPLE solve for {outer} outer iterations on {rec['threads']} threads ({dt:.0f} s).  Its start-up\n"
                f"solves (u0 = A^-1 f and the SIMPLE solve of g) took {rec['start_A']} A and {rec['start_S']} SIMPLE\n"
                f"inner iterations; the outer iterations took {per_outer_A} A and {per_outer_S} SIMPLE.  bench.py's\n"
                "CPU baseline multiplies these counts with the oracle's cost per inner iteration timed on the\n"
                "GPU box's host cores.\n\n```json\n")
        json.dump(rec, f, indent=1)
        f.write("\n```\n")
    log(f"[oracle-counts] {json.dumps(rec)}")


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def kernel_symbol(kind_name, precision):
    """The kernel symbol a timing kind names (the pipelined forms are FP64 only)."""
    if kind_name.endswith("_pipe"):
        return kind_name + "<double>"
    return kind_name


def cpu_baseline(workload, mask, gpu_rep, iters=30):
    """The oracle's cost per solve on the same geometry: its cost per inner A and
    per inner SIMPLE iteration, timed here on the host cores over a bounded run of
    each, times its own Jacobi inner iteration counts for this geometry (measured
    by --oracle-counts: the start-up solves, then the mean per outer iteration),
    times the outer iterations of the solve (the GPU's count; the oracle's agrees
    within one in every parity case).  None when no stored counts match."""
    import numpy as np
    import oracle
    path = oracle_counts_path(workload)
    try:
        rec = read_json_block(path)
    except (OSError, ValueError):
        log(f"[bench] no oracle inner counts at {path}; cpu_baseline omitted")
        return None
    if rec.get("mask_sha256_16") != _sha16(np.ascontiguousarray(mask).tobytes()) or \
            rec.get("oracle_c_sha256_16") != oracle_source_hash():
        log("[bench] stored oracle inner counts are for another geometry or oracle; cpu_baseline omitted")
        return None
    N = mask.shape[0]
    t0 = time.perf_counter()
    o = oracle.Oracle(mask, (1.0, 0.0, 0.0))
    t_asm = time.perf_counter() - t0
    f = np.zeros((3, N, N, N))
    f[0] = o.apply(oracle.OP_DIAG_A, None)[0] > 0
    t0 = time.perf_counter()
    _, itA = o.inner_solve(0, f, eps=1e-300, maxit=iters)
    itA = abs(itA) if itA >= 0 else -itA - 1
    tA = (time.perf_counter() - t0) / max(itA, 1)
    b = o.apply(oracle.OP_B, np.random.default_rng(0).standard_normal((3, N, N, N)))
    t0 = time.perf_counter()
    _, itS = o.inner_solve(1, b, eps=1e-300, maxit=iters)
    itS = abs(itS) if itS >= 0 else -itS - 1
    tS = (time.perf_counter() - t0) / max(itS, 1)
    mA = float(np.mean(rec["per_outer_A"]))
    mS = float(np.mean(rec["per_outer_S"]))
    outer = gpu_rep["outer_iters"]
    nA = rec["start_A"] + outer * mA
    nS = rec["start_S"] + outer * mS
    est = nA * tA + nS * tS
    return {
        "value": 1.0 / est, "unit": "solves/s", "cores": oracle.threads(), "kind": "oracle",
        "sample": (f"oracle (FP64, CSR over the active unknowns, Jacobi-PCG inner solves) on the same {N}^3 "
                   f"geometry: {itA} inner A iterations ({tA * 1e3:.1f} ms each) and {itS} inner SIMPLE "
                   f"iterations ({tS * 1e3:.1f} ms each) timed here; its own inner counts for this geometry "
                   f"({rec['start_A']} A + {rec['start_S']} SIMPLE to start, then {mA:.0f} A + {mS:.0f} SIMPLE "
                   f"per outer iteration, from its first {rec['outer_done']} outer iterations: "
                   f"profiles/{os.path.basename(path)}) times the {outer} outer iterations of this solve = "
                   f"{nA:.0f} A + {nS:.0f} SIMPLE iterations, {est:.0f} s per solve (assembly {t_asm:.1f} s and "
                   f"outer-loop vector work not counted); host {host_cpu_model()}, {os.cpu_count()} logical CPUs"),
        "seconds_per_solve_est": est,
    }


def large_solve(P, torch, workload="grf512"):
    """One mixed-precision SIMPLE solve of a large workload (setup reported
    beside the solve time, not in it)."""
    desc, N, gen = WORKLOADS[workload]
    log(f"[large] generating {desc}")
    t0 = time.perf_counter()
    mask = gen()
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    s = P.Stokes(mask, (1.0, 0.0, 0.0), stream=torch.cuda.current_stream().cuda_stream)
    s.set_option("precision", 1)
    s.set_option("progress", 40)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    info = s.info()
    del mask
    t0 = time.perf_counter()
    rep = s.solve(P.STOKES_SIMPLE, 1e-8)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s.close()
    log(f"[large] {desc}: mixed solve {dt:.2f} s outer={rep['outer_iters']} k={rep['k_hat']:.12e}")
    return {"workload": f"mixed FP32/FP64 SIMPLE solve, {desc}, force x, tol 1e-8", "N": N,
            "solve_s": dt, "solves_per_s": 1.0 / dt, "setup_s": t_setup, "generate_s": t_gen,
            "outer_iters": rep["outer_iters"], "inner_A_iters": rep["inner_A_iters"],
            "inner_S_iters": rep["inner_S_iters"], "k_hat": rep["k_hat"], "rel_res": rep["rel_res"],
            "div_norm": rep["div_norm"], "status": rep["status"], "porosity_effective": rep["porosity_effective"],
            "components_kept": info["ncomp_kept"]}


def generate_requests(n):
    """Masks of the first n serving requests, generated in worker processes
    (before this process touches the GPU)."""
    import multiprocessing as mp

    from synth.requests import make_request
    if n == 0:
        return []
    t0 = time.perf_counter()
    procs = max(1, min(16, os.cpu_count() or 1, n))
    with mp.get_context("fork").Pool(procs) as pool:
        reqs = pool.map(make_request, range(n), chunksize=1)
    log(f"[serve] generated {n} request geometries in {time.perf_counter() - t0:.1f} s on {procs} processes")
    return reqs


def collect(srv, ids, phase):
    """Results of the given requests, in order, with a line every 100 results."""
    res = []
    for q, i in enumerate(ids):
        res.append(srv.wait(i))
        if (q + 1) % 100 == 0 or q + 1 == len(ids):
            log(f"[serve] {phase}: {q + 1}/{len(ids)} results at t={res[-1]['t_end']:.1f} s")
    return res


def serve(P, reqs, slots=SERVE_SLOTS, budget=SERVE_BUDGET, frac=0.8, seed=12345, max_members=32):
    """Saturated throughput from the whole request stream submitted at once,
    then the same stream with Poisson arrivals at frac of that rate; latency =
    result ready - submitted.  max_members: requests per batched context (1:
    every request on a context of its own)."""
    import numpy as np

    with P.Server(slots, budget, max_members=max_members) as srv:
        t0 = srv.clock()
        ids = [srv.submit(m, precision=1) for _, m in reqs]
        res = collect(srv, ids, "saturated")
        mu = len(reqs) / (max(r["t_end"] for r in res) - t0)
        sat_stats = srv.stats()
        log(f"[serve] saturated: {len(reqs)} requests in {len(reqs) / mu:.2f} s -> {mu:.2f} requests/s")
        rate = frac * mu
        gaps = np.random.default_rng(seed).exponential(1.0 / rate, len(reqs))
        arrivals = np.cumsum(gaps) - gaps[0]
        start = time.perf_counter()
        ids = []
        for q, (_, m) in enumerate(reqs):
            delay = start + arrivals[q] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            ids.append(srv.submit(m, precision=1))
            if (q + 1) % 100 == 0:
                log(f"[serve] submitted {q + 1}/{len(reqs)}; {srv.stats()['completed']} done")
        res = collect(srv, ids, "poisson")
        stats = srv.stats()
    lat = np.array([r["t_end"] - r["t_submit"] for r in res])
    span = max(r["t_end"] for r in res) - min(r["t_submit"] for r in res)
    cells = sum(p["N"] ** 3 for p, _ in reqs)
    bad = [r for r in res if r["status"] != 0]
    return {
        "requests": len(reqs), "slots": slots, "hbm_budget_GB": budget / 2 ** 30,
        "precision": "mixed", "precond": "simple", "tol": 1e-8,
        "saturated_requests_per_s": mu, "saturated_voxels_per_s": mu * sum(p["N"] ** 3 for p, _ in reqs) / len(reqs),
        "arrival_rate_per_s": rate, "arrival_frac": frac,
        "throughput_requests_per_s": len(reqs) / span,
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3),
                       "mean": float(lat.mean() * 1e3), "max": float(lat.max() * 1e3)},
        "queue_wait_ms_p50": float(np.percentile([r["t_start"] - r["t_submit"] for r in res], 50) * 1e3),
        "peak_running": stats["peak_running"], "peak_bytes_GB": stats["peak_bytes"] / 2 ** 30,
        "voxels_per_s": cells / span, "failed": len(bad),
        "max_members_per_context": max_members,
        "saturated_requests_per_context": sat_stats["requests_on_contexts"] / max(1, sat_stats["contexts"]),
        "poisson_requests_per_context": (stats["requests_on_contexts"] - sat_stats["requests_on_contexts"]) /
                                        max(1, stats["contexts"] - sat_stats["contexts"]),
        "workload": "seeded request stream: spheres r 2..6 or GRF corr length 4..12 (50/50), N in "
                    "{32,48,64,96,128}, porosity 0.15..0.6, force x",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="tight256", choices=sorted(WORKLOADS),
                    help="geometry: the 256^3 tight sphere pack (default), the 128^3 spheres or the 512^3 field")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the mixed-precision 512^3 solve reported beside the line")
    ap.add_argument("--oracle-counts", action="store_true",
                    help="CPU only: measure the oracle's own inner iteration counts on --workload for the "
                         "CPU baseline and store them under profiles/")
    ap.add_argument("--precond", default="simple", choices=["simple", "uzawa"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--mixed-steps", type=int, default=3,
                    help="timed mixed-precision solves reported beside the FP64 line (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep-blocks", type=int, default=0)
    ap.add_argument("--max-outer", type=int, default=0,
                    help="cap the outer iterations (short runs for hardware-counter profiles)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 2 GiB device copy (reference for the byte counters; larger than "
                         "the 256 MB Infinity Cache)")
    ap.add_argument("--requests", type=int, default=48,
                    help="serving requests run beside the solve benchmark (0 = skip)")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving workload")
    ap.add_argument("--serve-slots", type=int, default=SERVE_SLOTS)
    ap.add_argument("--serve-members", type=int, default=32,
                    help="requests per batched context in the server (1 = no batching)")
    ap.add_argument("--study", choices=["precond", "precond256", "batch", "slits"],
                    help="instead of the benchmark: SIMPLE against Uzawa over 128^3 geometries (precond), or "
                         "batched contexts against one context per request for small boxes (batch)")
    args = ap.parse_args()
    if args.oracle_counts:
        measure_oracle_counts(args.workload)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    # one hardware queue per server slot; read when the process first uses HIP
    os.environ.setdefault("GPU_MAX_HW_QUEUES", str(max(4, args.serve_slots)))
    reqs = generate_requests(args.requests) if not args.study else []

    import torch

    import paper_2307_05266_amd as P
    from paper_2307_05266_amd.stokes import KERNEL_NAMES

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    P.load()
    if args.study == "precond":
        precond_study(P)
        return
    if args.study == "precond256":
        # the 256^3 tight pack: SIMPLE (the headline solve) against Uzawa
        precond_study(P, [(WORKLOADS["tight256"][0], WORKLOADS["tight256"][2])])
        return
    if args.study == "batch":
        batch_study(P, torch)
        return
    if args.study == "slits":
        slit_study(P, torch)
        return
    if args.serve_only:
        sv = serve(P, reqs, slots=args.serve_slots, max_members=args.serve_members)
        out = {"metric": "permeability solves/s (serving)", "value": sv["throughput_requests_per_s"],
               "unit": "solves/s", "n_gpus": 1, "higher_is_better": True, "vs_baseline": None,
               "dtype": "f32+f64", "data": "synthetic", "config": {"workload": sv["workload"]}, "serving": sv}
        print(json.dumps(out), flush=True)
        return
    desc, N, gen = WORKLOADS[args.workload]
    log(f"[bench] generating {desc}")
    mask = gen()
    pc = P.STOKES_SIMPLE if args.precond == "simple" else P.STOKES_UZAWA

    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    s = P.Stokes(mask, (1.0, 0.0, 0.0), stream=stream.cuda_stream)
    if N > 128:
        s.set_option("progress", 25)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    if args.sweep_blocks:
        s.set_option("sweep_blocks", args.sweep_blocks)
    if args.precision == "mixed":
        s.set_option("precision", 1)
    if args.max_outer:
        s.set_option("max_outer", args.max_outer)
    if args.copy_calibration:
        # 2 GiB read + 2 GiB written per copy, far beyond the 256 MB Infinity Cache
        src = torch.ones(256 * 2 ** 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    info = s.info()
    log(f"[bench] setup {setup_ms:.1f} ms, fluid {info['nfluid']} components {info['ncomp_kept']}")

    for w in range(args.warmup):
        rep = s.solve(pc, 1e-8)
        log(f"[bench] warmup {w}: {rep['seconds']:.3f} s outer={rep['outer_iters']} "
            f"innerA={rep['inner_A_iters']} innerS={rep['inner_S_iters']} k={rep['k_hat']:.10e}")

    s.set_option("kernel_timing", 32)   # time every 32nd iteration of each inner solve (the rest replay graphs)
    for kind in range(len(KERNEL_NAMES)):
        s.kernel_timing(kind)  # reset
    lat = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        t1 = time.perf_counter()
        rep = s.solve(pc, 1e-8)
        kh = s.permeability()
        lat.append(time.perf_counter() - t1)
        log(f"[bench] step {k}: {lat[-1]:.3f} s outer={rep['outer_iters']} k={kh:.12e}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    kernels = {}
    for kind, name in enumerate(KERNEL_NAMES):
        ms, n, nbytes = s.kernel_timing(kind)
        if n == 0:
            continue
        avg = ms / n
        kernels[name] = {"ms_total": ms, "launches": n, "avg_launch_us": avg * 1e3,
                         "bytes_per_launch": nbytes, "GBps": nbytes / (avg * 1e-3) / 1e9}
    s.set_option("kernel_timing", 0)
    copy_gbps = stream_copy_gbps(torch)
    log(f"[bench] plain device copy: {copy_gbps:.0f} GB/s")
    dom = max(kernels, key=lambda k: kernels[k]["ms_total"])
    achieved = kernels[dom]["GBps"]
    lat_sorted = sorted(lat)

    def pct(q):
        idx = min(len(lat_sorted) - 1, max(0, int(round(q * (len(lat_sorted) - 1)))))
        return lat_sorted[idx] * 1e3

    # inner iterations per solve and derived rates
    sweeps_A = rep["inner_A_iters"]
    sweeps_S = rep["inner_S_iters"]
    value = args.steps / total

    out = {
        "metric": "permeability solves/s",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{'FP64' if args.precision == 'fp64' else 'mixed FP32/FP64'} {args.precond.upper()} solve, "
                         f"{desc}, force x, tol 1e-8"),
            "N": N, "precond": args.precond, "precision": args.precision, "tol": 1e-8,
        },
        "latency_ms": {"p50": pct(0.5), "p99": pct(0.99)},
        "k_hat": rep["k_hat"],
        "div_norm": rep["div_norm"],
        "outer_iters": rep["outer_iters"],
        "inner_A_iters": sweeps_A,
        "inner_S_iters": sweeps_S,
        "setup_ms": setup_ms,
        "cell_updates_per_s": (sweeps_A + sweeps_S) * N ** 3 * args.steps / total,
        # the same over active unknowns only (faces for A, fluid cells for SIMPLE)
        "active_dof_updates_per_s": (sweeps_A * (info["nface_x"] + info["nface_y"] + info["nface_z"]) +
                                     sweeps_S * info["nfluid"]) * args.steps / total,
        "roofline": {
            "kernel": dom,
            # the code object that ran for that sweep (as rocprofv3 names it)
            "symbol": kernel_symbol(dom, args.precision),
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(dom, N),
            "launches": kernels[dom]["launches"],
            "avg_launch_us": kernels[dom]["avg_launch_us"],
            "bytes_per_launch": kernels[dom]["bytes_per_launch"],
            # a plain 1 GiB device copy on the same GPU in the same run: what
            # streaming reaches in practice, beside the published peak
            "stream_copy_GBps": copy_gbps,
            "frac_of_copy": achieved / copy_gbps,
        },
        "kernels": kernels,
    }
    if args.precision == "fp64" and args.mixed_steps > 0:
        # the same solve with FP32 inner solves and FP64 outer recurrences
        k64, div64 = rep["k_hat"], rep["div_norm"]
        s.set_option("precision", 1)
        if args.warmup > 0:
            rm = s.solve(pc, 1e-8)  # warm-up (allocates the FP32 vectors)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.mixed_steps):
            rm = s.solve(pc, 1e-8)
        torch.cuda.synchronize()
        tm = (time.perf_counter() - t0) / args.mixed_steps
        out["mixed_vs_fp64"] = {
            "value": 1.0 / tm, "unit": "solves/s", "ms_per_solve": tm * 1e3,
            "speedup_vs_fp64": (1.0 / tm) / value,
            "k_hat": rm["k_hat"], "k_rel_diff_vs_fp64": abs(rm["k_hat"] - k64) / abs(k64),
            "div_norm": rm["div_norm"], "div_norm_fp64": div64, "rel_res": rm["rel_res"],
            "outer_iters": rm["outer_iters"], "inner_A_iters": rm["inner_A_iters"],
            "inner_S_iters": rm["inner_S_iters"],
        }
        log(f"[bench] mixed: {tm:.3f} s/solve outer={rm['outer_iters']} k={rm['k_hat']:.12e}")
    s.close()
    if not args.no_large and args.workload != "grf512":
        out["large_mixed_solve"] = large_solve(P, torch)
    if reqs:
        out["serving"] = serve(P, reqs, slots=args.serve_slots, max_members=args.serve_members)
        log(f"[serve] {out['serving']['throughput_requests_per_s']:.2f} requests/s, latency p50 "
            f"{out['serving']['latency_ms']['p50']:.0f} ms p99 {out['serving']['latency_ms']['p99']:.0f} ms")
    if not args.no_cpu_baseline and N <= 256:
        log("[bench] timing the oracle on a bounded sample")
        cb = cpu_baseline(args.workload, mask, rep)
        if cb:
            out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
            out["cpu_baseline_seconds_per_solve_est"] = cb["seconds_per_solve_est"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
