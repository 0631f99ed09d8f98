#!/usr/bin/env python3
"""Benchmark of the HPS direct solver's hot path on one MI355X.

Workload (the problem the headline metric is quoted on): Omega = [0,1]^2 split into
64 x 64 leaves, p = 16 Chebyshev points per direction per leaf (DOF = 4096 * 252 =
1,032,192), kappa = eta = 100, c(x,y) = 1 - 0.5 exp(-160((x-.5)^2 + (y-.5)^2)),
complex128.  The 16 right-hand sides of one solve call are manufactured from
u = exp(i kappa d.x)(1 + 0.1 sin 2 pi x sin 2 pi y) with seeded unit directions d.

A step is one pass of the whole hot path: hps_build (batched leaf stage + every merge
level) followed by one 16-RHS hps_solve (upward + downward sweeps), inputs resident in
HBM.  Prints one JSON line (see the keys below).

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

METRIC = "HPS build DOF/s + RHS solves/s at stated rel. L2 error; p99 solve latency"
PEAK = {"hbm": (8000.0, "GB/s"), "mfma": (78.6, "TFLOP/s"), "mfma32": (157.3, "TFLOP/s"),
        "alu": (78.6, "TFLOP/s")}


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from a committed profiler summary under profiles/
    (two counter passes scaled by a plain copy), or None when there is none or the
    kernel's source file has changed since it was measured."""
    import glob
    import hashlib
    for fn in glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md")):
        kv = {}
        for line in open(fn):
            if " = " in line:
                k, v = line.strip().split(" = ", 1)
                kv[k] = v
        if kv.get("kernel") != kernel or "kernel_source" not in kv:
            continue
        src = os.path.join(ROOT, kv["kernel_source"])
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest() if os.path.exists(src) else ""
        if kv.get("kernel_source_sha256") == sha:
            return float(kv["traffic_bytes_per_launch"])
    return None


def kernel_of(stage, p):
    """The kernel function behind a timing record of the library, with its roofline
    bound, or None when the record covers several kernels.  The GEMM's tile variants are
    instances of one kernel template and count as one kernel: which variant a shape gets
    is the autotuner's timing-dependent choice."""
    import re
    base = stage.split("@")[0].split("[")[0]
    if "[" in stage:
        var = stage[stage.index("[") + 1:-1]
        mt = re.fullmatch(r"(\d+x\d+)([rc])([rc])(s?)", var)
        if mt.group(4):  # complex64 operands on the FP32 matrix cores
            return "zgemm_kernel<float, ...> (every tile variant)", "mfma32"
        return "zgemm_kernel<double, ...> (every tile variant)", "mfma"
    return {"leaf_sinv": ("leaf_sinv_kernel<%d>" % p, "alu"),
            "leaf_psi_bnd": ("leaf_psi_bnd_kernel<%d>" % p, "hbm"),
            "leaf_ainv": ("leaf_ainv_kernel<%d>" % p, "alu"),
            "leaf_xz": ("leaf_xz_kernel<%d>" % p, "hbm")}.get(base)


def merge_levels(nx, ny, p):
    """(nbox, n1, n2, n3) per merge level, root first: the tree splits a box of wx x wy
    leaves across its longer side (ties split x); the shared edge holds n3 nodes and the
    children's outer boundaries n1 and n2."""
    m = p - 2
    out, boxes = [], [(nx, ny)]
    while boxes and max(max(b) for b in boxes) > 1:
        nxt, lev = [], []
        for wx, wy in boxes:
            split_x = True if wy == 1 else False if wx == 1 else wx >= wy
            if split_x:
                c = (wx // 2, wy)
                n3 = wy * m
            else:
                c = (wx, wy // 2)
                n3 = wx * m
            n1 = 2 * (c[0] + c[1]) * m - n3
            lev.append((n1, n1, n3))
            nxt += [c, c]
        out.append((len(boxes),) + lev[0])
        boxes = nxt
    return out


def survey_work(nx, ny, p, nrhs):
    """Algorithmic work of one step by the survey's per-unit formulas (Sec. 8(d)): the leaf
    stage F_leaf per leaf (real c, block elimination, Psi and Y formed), the merge stage
    F_merge per merge (LU-count interface solve, no explicit-inverse flops), and the bytes
    of one solve call with a body load (operators read once, s and u moved once)."""
    m = p - 2
    ni, nb, n = m * m, 4 * m, p * p - 4
    nleaf = nx * ny
    f_leaf = 2 * ni ** 3 + 8 * ni ** 2 * nb + 2 * nb ** 2 * ni + 8 * nb ** 3 + 8 * ni * nb ** 2
    f_merge, ops_merge = 0.0, 0.0
    for nbox, n1, n2, n3 in merge_levels(nx, ny, p):
        f_merge += nbox * (8 * n3 ** 3 + 8.0 / 3.0 * n3 ** 3 + 8 * n3 ** 2 * n1 +
                           16 * n3 ** 2 * (n1 + n2) + 8 * n3 * (n1 + n2) ** 2)
        ops_merge += nbox * (3 * n3 ** 2 + 3 * n3 * (n1 + n2))
    solve_bytes = 16.0 * (nleaf * n * n + ops_merge + nrhs * nleaf * (ni + n))
    return {"F_leaf_per_leaf": f_leaf, "F_leaf": f_leaf * nleaf, "F_merge": f_merge,
            "solve_bytes": solve_bytes}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(nx=64, ny=64, p=16, kappa=100.0, nrhs=16, seed=0, nodes=None):
    from paper_1812_07167_amd import inputs as G
    xy, xyi, xyb, nrm = nodes(nx, ny, p)
    c = G.c_gaussian_bump(xyi)
    thetas = G.seeded_thetas(seed, nrhs)
    mfs = [G.Manufactured(kappa, float(a)) for a in thetas]
    s = np.stack([mf.s(xyi, c) for mf in mfs])
    t = np.stack([mf.t(xyb, nrm, kappa) for mf in mfs])
    exact = np.stack([mf.u(xy) for mf in mfs])
    return c, s, t, exact


def host_cpu():
    """The host processor's model name (first entry of /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(nx, ny, p, kappa, nrhs, seed):
    """The CPU oracle, as it stands, on a bounded sample of the workload: the corner
    [0, nx/64] x [0, ny/64] of the unit square with the workload's own 1/64 x 1/64 leaves,
    the same p, kappa, c and manufactured right-hand sides."""
    from oracle import hps_oracle as O
    x1, y1 = nx / 64.0, ny / 64.0

    def onodes(a, b, pp):
        prob = O.Problem(0.0, x1, 0.0, y1, a, b, pp, kappa, kappa)
        bd, nr = prob.root_boundary()
        return prob.leaf_nodes(), prob.interior_nodes(), bd, nr

    c, s, t, exact = workload(nx, ny, p, kappa, nrhs, seed, onodes)
    prob = O.Problem(0.0, x1, 0.0, y1, nx, ny, p, kappa, kappa)
    t0 = time.perf_counter()
    boxes = O.build(prob, c)
    u = O.solve(prob, boxes, s, t)
    dt = time.perf_counter() - t0
    cores = os.cpu_count()
    try:
        from threadpoolctl import threadpool_info
        nth = [i.get("num_threads") for i in threadpool_info() if i.get("user_api") == "blas"]
        if nth:
            cores = int(max(nth))
    except Exception:
        pass
    dof = nx * ny * (p * p - 4)
    err = float(np.linalg.norm(u - exact) / np.linalg.norm(exact))
    return {"value": dof / dt, "unit": "DOF/s (build + one %d-RHS solve)" % nrhs, "cores": cores,
            "kind": "oracle", "seconds": dt, "rel_l2_vs_exact": err, "host_cpu": host_cpu(),
            "host_cpus_visible": os.cpu_count(),
            "sample": "oracle build + one %d-RHS solve on the %dx%d-leaf corner [0,%g]x[0,%g] "
                      "of the workload (same leaves, p=%d, kappa=%g, c and right-hand "
                      "sides; %.3g of its DOF); numpy/OpenBLAS, threads as counted"
                      % (nrhs, nx, ny, x1, y1, p, kappa, nx * ny / 4096.0)}


def mixed_leg(H, torch, dom, p, kappa, c_d, s_d, t_d, u_ref, exact, stream, out, reps=3):
    """The same build + 16-RHS solve with complex64 merges and solve products (FP64
    leaves, top-3-level interface inverses and residual correction), against the
    complex128 result."""
    u_c128 = u_ref.clone()
    u = torch.empty_like(u_ref)
    f = H.hps_build(dom, p, kappa, kappa, c_d, stream=stream, precision=H.HPS_PREC_MIXED,
                    autotune=True)
    H.hps_solve(f, t_d, s_d, u)
    f.free()
    torch.cuda.synchronize()
    bms, sms = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        f = H.hps_build(dom, p, kappa, kappa, c_d, stream=stream, precision=H.HPS_PREC_MIXED)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        H.hps_solve(f, t_d, s_d, u)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        it, conv, corr = f.last_solve_info()
        f.free()
        bms.append((t1 - t0) * 1e3)
        sms.append((t2 - t1) * 1e3)
    um, uc = u.cpu().numpy(), u_c128.cpu().numpy()
    b, s_ = float(np.median(bms)), float(np.median(sms))
    return {"build_ms": round(b, 3), "solve_ms": round(s_, 3),
            "correction_steps": it, "converged": conv, "last_relative_correction": corr,
            "rel_l2_vs_c128": float(np.linalg.norm(um - uc) / np.linalg.norm(uc)),
            "rel_l2_vs_exact": float(np.linalg.norm(um - exact) / np.linalg.norm(exact)),
            "build_speedup_vs_c128": round(out["build_ms"] / b, 3),
            "solve_speedup_vs_c128": round(out["solve_ms"] / s_, 3),
            "fp64_top_levels": 3}


def precision_leg(H, torch, dev, stream, nx=128, p=16, kappa=300.0, nrhs=4, seed=4, reps=2):
    """The precision comparison at scale: 128 x 128 leaves, p = 16 (4.1M collocation
    nodes), kappa = eta = 300, Fourier c, manufactured right-hand sides with seeded
    directions.  The complex128 build + solve against the mixed one (complex64 merges and
    solve products on the FP32 matrix cores, FP64 leaves, top-3-level interface inverses
    and residual correction): times, error against the closed form and against
    complex128."""
    from paper_1812_07167_amd import inputs as G
    dom = H.domain(nx, nx)
    xy, xyi, xyb, nrm = H.hps_nodes(dom, p)
    c = G.FourierField.seeded(seed)(xyi)
    mfs = [G.Manufactured(kappa, float(a)) for a in G.seeded_thetas(seed, nrhs)]
    s_d = torch.tensor(np.stack([mf.s(xyi, c) for mf in mfs]), dtype=torch.complex128, device=dev)
    t_d = torch.tensor(np.stack([mf.t(xyb, nrm, kappa) for mf in mfs]), dtype=torch.complex128,
                       device=dev)
    exact = np.stack([mf.u(xy) for mf in mfs])
    c_d = torch.tensor(c, dtype=torch.float64, device=dev)
    dof = nx * nx * (p * p - 4)
    out = {"leaves": nx * nx, "p": p, "kappa": kappa, "dof": dof, "nrhs": nrhs}
    sols = {}
    for name, prec in (("c128", H.HPS_PREC_C128), ("mixed", H.HPS_PREC_MIXED)):
        bms, sms = [], []
        for r in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f = H.hps_build(dom, p, kappa, kappa, c_d, stream=stream, precision=prec,
                            autotune=(r == 0))
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            u = H.hps_solve(f, t_d, s_d)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            info = f.last_solve_info()
            f.free()
            bms.append((t1 - t0) * 1e3)
            sms.append((t2 - t1) * 1e3)
        sols[name] = u.cpu().numpy()
        del u
        err = float(np.linalg.norm(sols[name] - exact) / np.linalg.norm(exact))
        out[name] = {"build_ms": round(min(bms), 2), "solve_ms": round(min(sms), 2),
                     "build_dof_per_s": round(dof / (min(bms) * 1e-3), 1),
                     "rel_l2_vs_exact": err,
                     "factor_gb": round(H.hps_estimate_bytes(dom, p, precision=prec)[1] / 1e9, 2)}
        if prec == H.HPS_PREC_MIXED:
            out[name]["correction_steps"] = info[0]
            out[name]["last_relative_correction"] = info[2]
    out["mixed"]["rel_l2_vs_c128"] = float(np.linalg.norm(sols["mixed"] - sols["c128"]) /
                                          np.linalg.norm(sols["c128"]))
    out["build_speedup_mixed"] = round(out["c128"]["build_ms"] / out["mixed"]["build_ms"], 3)
    out["solve_speedup_mixed"] = round(out["c128"]["solve_ms"] / out["mixed"]["solve_ms"], 3)
    return out


def batch_leg(H, torch, dev, stream, count=256, seed0=0, reps=2):
    """Cross-problem batching: `count` independent seeded problems (leaf grids 8^2..32^2,
    p in {8, 12, 16}, kappa in [10, 80], Fourier c, one manufactured right-hand side each)
    built with hps_build_batch and solved with hps_solve_batch, in complex128 and in mixed
    precision, against the same problems built and solved one at a time."""
    from paper_1812_07167_amd import inputs as G
    probs = G.batch_problems(seed0, count)
    nodes = {}
    doms, ps, ks, cs, ss, ts, exact = [], [], [], [], [], [], []
    dof = 0
    for q in probs:
        key = (q["nx"], q["p"])
        if key not in nodes:
            nodes[key] = H.hps_nodes(H.domain(q["nx"], q["ny"]), q["p"])
        xy, xyi, xyb, nrm = nodes[key]
        c = G.FourierField.seeded(q["seed"])(xyi)
        mf = G.Manufactured(q["kappa"], q["theta"])
        doms.append(H.domain(q["nx"], q["ny"]))
        ps.append(q["p"])
        ks.append(q["kappa"])
        cs.append(torch.tensor(c, dtype=torch.float64, device=dev))
        ss.append(torch.tensor(mf.s(xyi, c)[None], dtype=torch.complex128, device=dev))
        ts.append(torch.tensor(mf.t(xyb, nrm, q["kappa"])[None], dtype=torch.complex128,
                               device=dev))
        exact.append(mf.u(xy))
        dof += q["nx"] * q["ny"] * (q["p"] ** 2 - 4)
    # one factorization group per shape; the groups' launch chains run side by side on
    # up to four streams of the library
    res = {"problems": count, "dof": dof, "shape_groups": len(nodes),
           "launch_chains_per_merge_level": len(nodes), "groups_built_at_once": min(4, len(nodes)),
           "max_rel_l2_vs_exact_note": "discretization error of the worst drawn problem "
                                       "(kappa up to 80 on 8x8 leaves of p = 8, under-resolved)"}

    def run(precision):
        bt, st_ = [], []
        for rep in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            # the first repetition tunes the GEMM shapes it meets (the minimum is reported)
            fs = H.hps_build_batch(doms, ps, ks, ks, cs, stream=stream, precision=precision,
                                   autotune=(rep == 0))
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            us = H.hps_solve_batch(fs, ts, ss)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            bt.append((t1 - t0) * 1e3)
            st_.append((t2 - t1) * 1e3)
            for f in fs:
                f.free()
        sol = [u.cpu().numpy()[0] for u in us]
        errs = [float(np.linalg.norm(u - e) / np.linalg.norm(e)) for u, e in zip(sol, exact)]
        b, s_ = float(np.min(bt)), float(np.min(st_))
        return sol, {"build_ms": round(b, 2), "solve_ms": round(s_, 2),
                     "build_dof_per_s": round(dof / (b * 1e-3), 1),
                     "rhs_solves_per_s": round(count / (s_ * 1e-3), 1),
                     # discretization error: some drawn problems (kappa up to 80 on 8 x 8
                     # leaves of p = 8) are under-resolved on purpose
                     "median_rel_l2_vs_exact": float(np.median(errs)),
                     "max_rel_l2_vs_exact": float(np.max(errs))}

    sol128, res["c128"] = run(H.HPS_PREC_C128)
    solmx, res["mixed"] = run(H.HPS_PREC_MIXED)
    res["mixed"]["max_rel_l2_vs_c128"] = max(
        float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(solmx, sol128))
    # the same problems one at a time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(count):
        f = H.hps_build(doms[i], ps[i], ks[i], ks[i], cs[i], stream=stream)
        H.hps_solve(f, ts[i], ss[i])
        f.free()
    torch.cuda.synchronize()
    seq = (time.perf_counter() - t0) * 1e3
    res["one_at_a_time_ms"] = round(seq, 2)
    res["batch_speedup_c128"] = round(seq / (res["c128"]["build_ms"] + res["c128"]["solve_ms"]), 3)
    return res


def serve_leg(H, torch, dev, n_problems=32, n_requests=10000, load=0.7, slots=4,
              solve_slots=1, seed=0, max_rhs=64, new_build_every=100, reserve_gb=48.0,
              checks=64, headroom_gb=24.0, probe_requests=1000, window=64):
    """Serving: `n_problems` seeded problems (leaf grids 32^2..128^2, p 12-16, kappa
    50-300, Fourier c; complex128) built through the request loop under a device-memory
    budget of their resident bytes, plus the largest build's scratch, plus `headroom_gb`
    (less than concurrent solves' workspaces and new problems need at peaks, so that
    factors are evicted and rebuilt), then a Poisson stream of `n_requests` solve requests of 1..max_rhs
    right-hand sides each (smooth random s, plane-wave t) at `load` times the closed-loop
    saturated throughput of all slots, measured first under the same budget with
    `window` requests kept outstanding.  Every `new_build_every` requests a new problem
    is built and a live one of the same leaf grid released.  Latency is submission to completion.  `checks`
    seeded requests of the stream are re-solved alone on factors built outside the
    server and compared."""
    from paper_1812_07167_amd import inputs as G
    n_new = n_requests // new_build_every if new_build_every else 0
    probs = G.serve_problems(seed, n_problems + n_new)
    t_setup = time.perf_counter()
    data = []
    for q in probs:
        dom = H.domain(q["nx"], q["ny"])
        _, xyi, xyb, nrm = H.hps_nodes(dom, q["p"])
        c = G.FourierField.seeded(q["seed"])(xyi)
        f = torch.tensor(np.stack([G.FourierField.seeded(sd)(xyi) - 1.0 for sd in q["s_seeds"]]),
                         dtype=torch.complex128, device=dev)
        rng = np.random.default_rng(q["seed"] + 7)
        co = torch.tensor(rng.standard_normal((max_rhs, 2)) + 1j * rng.standard_normal((max_rhs, 2)),
                          dtype=torch.complex128, device=dev)
        S = co[:, 0:1] * f[0:1] + co[:, 1:2] * f[1:2]  # [max_rhs, n_interior], smooth
        th = G.seeded_thetas(q["seed"] + 11, max_rhs)
        T = np.stack([G.PlaneWave(q["kappa"], float(a)).t(xyb, nrm, q["kappa"]) for a in th])
        data.append({"dom": dom, "p": q["p"], "kappa": q["kappa"], "side": q["nx"],
                     "c": torch.tensor(c, dtype=torch.float64, device=dev),
                     "S": S.contiguous(), "T": torch.tensor(T, dtype=torch.complex128, device=dev),
                     "n": q["nx"] * q["ny"] * (q["p"] ** 2 - 4),
                     "est": H.hps_estimate_bytes(dom, q["p"])})
        del f, co
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    # memory cached by earlier legs (torch's and the library's) goes back to the device
    # before the budget is sized from what is free
    torch.cuda.empty_cache()
    H.hps_release_cached()
    free, total = torch.cuda.mem_get_info()
    # torch's own cache (inputs, and the outputs of outstanding requests, whose sizes
    # vary) stays within the reserve, so that the server's budget is device memory it
    # really has
    torch.cuda.set_per_process_memory_fraction(
        min(1.0, (torch.cuda.memory_allocated() + reserve_gb * 1e9) / total))
    resident = sum(d["est"][1] for d in data[:n_problems])
    scratch = max(d["est"][0] - d["est"][1] for d in data)
    budget = int(min(free * 0.9 - reserve_gb * 1e9, resident + scratch + headroom_gb * 1e9))
    srv = H.Server(budget_bytes=budget, slots=slots, solve_slots=solve_slots)
    res = {"problems": n_problems, "new_builds": n_new, "requests": n_requests,
           "max_rhs_per_request": max_rhs, "slots": slots, "solve_only_slots": solve_slots,
           "budget_gb": round(budget / 1e9, 2), "resident_estimate_gb": round(resident / 1e9, 2),
           "largest_build_scratch_gb": round(scratch / 1e9, 2),
           "setup_s": round(t_setup, 2)}
    rng_all = np.random.default_rng(seed + 2)
    outstanding, held = {}, [0]
    out_cap = reserve_gb * 1e9 * 0.5  # bytes of outputs of outstanding requests

    retries = [0]

    def out_bytes(nr, d):
        # outputs come from buckets of eight sizes per power of two (at most 1/8 wasted),
        # so that torch's cache reuses freed blocks instead of fragmenting over the many
        # request sizes
        n_el = nr * d["n"]
        q = 1 << max(0, (n_el - 1).bit_length() - 3)
        return -(-n_el // q) * q * 16

    def submit(pid, d, nr):
        n_el = nr * d["n"]
        cap = out_bytes(nr, d) // 16
        while True:
            try:
                buf = torch.empty(cap, dtype=torch.complex128, device=dev)
                break
            except torch.OutOfMemoryError:
                retries[0] += 1
                while outstanding and retries[0]:
                    drain(50)
                    if len(outstanding) < 8:
                        break
                torch.cuda.empty_cache()
        u = buf[:n_el].view(nr, d["n"])
        r, u = srv.solve(pid, d["T"][:nr], d["S"][:nr], u=u, sync=False)
        outstanding[r] = cap * 16
        held[0] += cap * 16
        return r, u

    def sample(u):
        # a strided sample of a result's entries and its norm (a kept request's output is
        # not held whole: 64 of them would take tens of GB)
        flat = u.reshape(-1)
        step = max(1, flat.numel() // 65536)
        return flat[::step].clone(), float(torch.linalg.norm(u))

    kept = {}

    # completions are recorded into the current phase's latency list and counters
    cur = {"lat": None, "counts": None}

    def drain(timeout_ms):
        lat, counts = cur["lat"], cur["counts"]
        for c in srv.poll(256, timeout_ms):
            if c["kind"] == H.HPS_REQ_SOLVE and c["req"] in outstanding:
                assert c["status"] == 0, c
                if c["req"] in kept:
                    di, nr, u = kept[c["req"]]
                    kept[c["req"]] = (di, nr, sample(u))
                held[0] -= outstanding.pop(c["req"])
                if lat is not None:
                    lat.append(c["t_end"] - c["t_submit"])
                if counts is not None:
                    counts[0] += 1
                    counts[1] += c["nrhs"]

    try:
        # builds of the resident set, all submitted at once
        t0 = time.perf_counter()
        built = [srv.build(d["dom"], d["p"], d["kappa"], d["kappa"], d["c"])
                 for d in data[:n_problems]]
        pids = [pid for pid, _ in built]
        bdone = srv.wait([req for _, req in built], timeout_s=600)
        assert all(c["status"] == 0 for c in bdone.values()), "a build failed"
        res["build_phase_s"] = round(time.perf_counter() - t0, 3)
        res["build_dof_per_s"] = round(sum(d["n"] for d in data[:n_problems]) / res["build_phase_s"], 1)
        log(f"serving: {n_problems} problems built in {res['build_phase_s']} s "
            f"(budget {res['budget_gb']} GB of {res['resident_estimate_gb']} GB resident)")
        # closed loop: `window` requests outstanding (fewer when their outputs would pass
        # the output cap) until probe_requests have completed
        live = list(zip(pids, range(n_problems)))  # (problem id, index into data)
        ppick, pnr, _ = G.poisson_requests(seed + 3, probe_requests + window, max_rhs)
        counts, k = [0, 0], 0
        cur["counts"] = counts
        t0 = time.perf_counter()
        while counts[0] < probe_requests:
            while len(outstanding) < window and k < len(ppick):
                pid, di = live[int(ppick[k] * len(live))]
                if outstanding and held[0] + out_bytes(int(pnr[k]), data[di]) > out_cap:
                    break
                submit(pid, data[di], int(pnr[k]))
                k += 1
            drain(20)
        t_probe = time.perf_counter() - t0
        done_probe, rhs_probe = counts
        cur["counts"] = None
        while outstanding:
            drain(100)
        sat = done_probe / t_probe
        rate = load * sat
        res["closed_loop_window"] = window
        res["saturated_req_per_s"] = round(sat, 2)
        res["saturated_rhs_per_s"] = round(rhs_probe / t_probe, 1)
        res["offered_rate_req_per_s"] = round(rate, 2)
        log(f"serving: closed-loop {sat:.1f} req/s; offering {rate:.1f} req/s")
        # the open-loop stream
        pick, nrhs, gaps = G.poisson_requests(seed + 1, n_requests, max_rhs)
        arrive = np.cumsum(gaps) / rate
        keep = set(rng_all.choice(n_requests, size=min(checks, n_requests), replace=False).tolist())
        nxt_new = n_problems
        lat, counts, backpressure, released = [], [0, 0], 0, 0
        cur["lat"], cur["counts"] = lat, counts
        st0 = srv.stats()
        t_start = time.perf_counter()
        for k in range(n_requests):
            if new_build_every and k > 0 and k % new_build_every == 0 and nxt_new < len(data):
                d = data[nxt_new]
                live.append((srv.build(d["dom"], d["p"], d["kappa"], d["kappa"], d["c"])[0],
                             nxt_new))
                nxt_new += 1
                # a live problem of the same leaf grid leaves (its queued requests still
                # complete), so the live set's memory stays about the same
                same = [i for i in range(len(live) - 1) if data[live[i][1]]["side"] == d["side"]]
                pool = same if same else list(range(len(live) - 1))
                gone = pool[int(rng_all.integers(len(pool)))]
                srv.release(live.pop(gone)[0])
                released += 1
            if k % 1000 == 0 and k:
                log(f"serving: {k} requests submitted, {counts[0]} done")
            pid, di = live[int(pick[k] * len(live))]
            d = data[di]
            nr = int(nrhs[k])
            # outputs of outstanding requests stay within the memory left beside the budget
            while held[0] + out_bytes(nr, d) > out_cap and outstanding:
                backpressure += 1
                drain(50)
            wait = t_start + arrive[k] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            r, u = submit(pid, d, nr)
            if k in keep:
                kept[r] = (di, nr, u)
            del u
            drain(0)
        while outstanding:
            drain(100)
        t_stream = time.perf_counter() - t_start
        st = srv.stats()
    finally:
        srv.close()
        torch.cuda.set_per_process_memory_fraction(1.0)
    lat = np.array(lat) * 1e3
    calls = st["batches"] - st0["batches"]
    sb = st["shared_batches"] - st0["shared_batches"]
    res.update({
        "stream_s": round(t_stream, 3),
        "solves_per_s": round(n_requests / t_stream, 2),
        "rhs_per_s": round(counts[1] / t_stream, 1),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3),
                       "max": round(float(lat.max()), 3)},
        "solve_calls": calls,
        "mean_rhs_per_solve_call": round((st["rhs"] - st0["rhs"]) / max(1, calls), 2),
        "shared_solve_calls": sb,
        "mean_problems_per_shared_call": round(
            (st["shared_problems"] - st0["shared_problems"]) / max(1, sb), 2),
        "evictions": st["evictions"] - st0["evictions"],
        "rebuilds": st["rebuilds"] - st0["rebuilds"],
        "evictions_total": st["evictions"], "rebuilds_total": st["rebuilds"],
        "released": released,
        "live_resident_estimate_gb_end": round(sum(data[di]["est"][1] for _, di in live) / 1e9, 2),
        "max_concurrent": st["max_concurrent"], "backpressure_waits": backpressure,
        "output_alloc_retries": retries[0],
        "retried_after_nomem": st["retried"] - st0["retried"],
        "peak_committed_gb": round(st["peak_committed_bytes"] / 1e9, 2),
    })
    # the kept requests solved alone, on factors built outside the server (one build per
    # problem they use)
    worst, worst_norm, by = 0.0, 0.0, {}
    for r, (di, nr, smp) in kept.items():
        by.setdefault(di, []).append((nr, smp))
    for di, items in by.items():
        d = data[di]
        f = H.hps_build(d["dom"], d["p"], d["kappa"], d["kappa"], d["c"])
        for nr, (us, un) in items:
            ua = H.hps_solve(f, d["T"][:nr], d["S"][:nr])
            torch.cuda.synchronize()
            uas, uan = sample(ua)
            worst = max(worst, float(torch.linalg.norm(us - uas) / torch.linalg.norm(uas)))
            worst_norm = max(worst_norm, abs(un - uan) / uan)
            del ua
        f.free()
    res["alone_vs_mix_max_rel_l2"] = worst
    res["alone_vs_mix_sample"] = ("every k-th entry of each kept result, about 65536 of them, "
                                  "plus the relative difference of the full norms")
    res["alone_vs_mix_max_norm_rel_diff"] = worst_norm
    res["alone_vs_mix_checked"] = len(kept)
    res["alone_vs_mix_problems"] = len(by)
    return res


def copy_calibration(torch, dev, mib=256, reps=3):
    """A plain device-to-device copy of `mib` MiB, `reps` times: the HBM byte counters
    of a profiler run over this command read what one copy of known size costs."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "reps": reps}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nrhs", type=int, default=16)
    ap.add_argument("--latency-solves", type=int, default=40)
    ap.add_argument("--cpu-leaves", default="64x32",
                    help="leaf grid of the oracle's sample of the workload (NXxNY)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the cross-problem batching leg (256 problems)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision (complex64 + FP64 correction) leg")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default GEMM tile choice (no tuning in the warmup build)")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the serving leg (request loop under a Poisson stream)")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="solve requests in the serving leg's stream")
    ap.add_argument("--serve-new-every", type=int, default=100,
                    help="requests between new builds in the serving stream (0: none)")
    ap.add_argument("--serve-reserve-gb", type=float, default=48.0,
                    help="device memory kept outside the server's budget for torch (inputs "
                         "and the outputs of outstanding requests)")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving leg (no step timing, no JSON line)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for scaling the HBM "
                         "byte counters of a profiler run) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1812_07167_amd import hps as H

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        copy_calibration(torch, dev)
        return
    H.load()
    if args.serve_only:
        print(json.dumps({"serving": serve_leg(H, torch, dev, n_requests=args.serve_requests,
                                   new_build_every=args.serve_new_every,
                                   reserve_gb=args.serve_reserve_gb)}))
        return
    nx = ny = 64
    p, kappa, nrhs = 16, 100.0, args.nrhs
    dom = H.domain(nx, ny)

    def lnodes(a, b, pp):
        return H.hps_nodes(H.domain(a, b), pp)

    c, s, t, exact = workload(nx, ny, p, kappa, nrhs, 0, lnodes)
    c_d = torch.tensor(c, dtype=torch.float64, device=dev)
    s_d = torch.tensor(s, dtype=torch.complex128, device=dev)
    t_d = torch.tensor(t, dtype=torch.complex128, device=dev)
    u_d = torch.empty((nrhs, nx * ny * (p * p - 4)), dtype=torch.complex128, device=dev)
    stream = torch.cuda.current_stream()
    dof = nx * ny * (p * p - 4)

    def step(profile, autotune=False):
        f = H.hps_build(dom, p, kappa, kappa, c_d, stream=stream, profile=profile,
                        autotune=autotune)
        tb = time.perf_counter()
        H.hps_solve(f, t_d, s_d, u_d)
        return f, tb

    # the first warmup build runs the GEMM autotuner (tile variants timed per merge
    # GEMM shape, the analog of the paper's per-level thread calibration); the timed
    # steps launch the recorded variants
    log("warmup", args.warmup)
    tune_s = None
    for w in range(args.warmup):
        t0 = time.perf_counter()
        f, _ = step(False, autotune=(w == 0 and not args.no_autotune))
        torch.cuda.synchronize()
        if w == 0:
            tune_s = time.perf_counter() - t0
        f.free()

    build_ms, solve_ms, step_ms = [], [], []
    torch.cuda.synchronize()
    t_all0 = time.perf_counter()
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f, tb = step(False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        build_ms.append((tb - t0) * 1e3)
        solve_ms.append((t1 - tb) * 1e3)
        step_ms.append((t1 - t0) * 1e3)
        f.free()
        log("step", k, "build %.2f ms solve %.2f ms" % (build_ms[-1], solve_ms[-1]))
    torch.cuda.synchronize()
    t_all1 = time.perf_counter()
    ms_per_step = (t_all1 - t_all0) * 1e3 / args.steps

    # the library's per-stage timing records (HIP events on the stream the kernels run
    # on) come from one more step with profiling on, outside the timed region (the
    # events add about 0.8 ms to a build and to a solve)
    f, _ = step(True)
    torch.cuda.synchronize()
    stages_b, stages_s = f.stage_times(0), f.stage_times(1)
    f.free()

    # accuracy of the last step's solution against the closed form
    u = u_d.cpu().numpy()
    err = float(np.linalg.norm(u - exact) / np.linalg.norm(exact))
    # e_inf of Sec. 4.1: the largest pointwise error at the collocation nodes
    einf = float(np.max(np.abs(u - exact)))

    # steady-state solve latency on one resident factor
    f = H.hps_build(dom, p, kappa, kappa, c_d, stream=stream)
    lat = []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        H.hps_solve(f, t_d, s_d, u_d)
    torch.cuda.synchronize()
    for _ in range(args.latency_solves):
        t0 = time.perf_counter()
        H.hps_solve(f, t_d, s_d, u_d)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)
    f.free()
    lat = np.array(lat)

    # roofline of the dominant kernel: the kernel with the largest summed time in a
    # step, among the timing records that each cover launches of one kernel only
    groups, kernels = {}, {}
    for name, launches, ms, fl, by in list(stages_b) + list(stages_s):
        base = name.split("@")[0].split("[")[0]
        g = groups.setdefault(base, [0, 0.0, 0.0, 0.0])
        g[0] += launches
        g[1] += ms
        kb = kernel_of(name, p)
        if kb is not None:
            kk = kernels.setdefault(kb, [0, 0.0, 0.0, 0.0])
            kk[0] += launches
            kk[1] += ms
            kk[2] += fl
            kk[3] += by
    (kname, bound), (launches, ms, fl, by) = max(kernels.items(), key=lambda kv: kv[1][1])
    peak, unit = PEAK[bound]
    if bound == "hbm":
        achieved = by / (ms * 1e-3) / 1e9
        per_launch = by / launches
    else:
        achieved = fl / (ms * 1e-3) / 1e12
        per_launch = fl / launches
    roofline = {"bound": "mfma" if bound == "mfma32" else bound, "achieved": round(achieved, 3),
                "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": measured_traffic(kname),
                "kernel": kname, "launches_per_step": launches,
                "avg_launch_ms": round(ms / launches, 5),
                "algorithmic_per_launch": per_launch,
                "algorithmic_unit": "bytes" if bound == "hbm" else "flops",
                "algorithmic_bytes_per_launch": by / launches}

    # stage-level roofline fractions by the survey's algorithmic work (Sec. 8(d)): the leaf
    # stage (F_leaf), the merge stage (F_merge over W, its LU-count solve, Phi and R^tau;
    # gathers included in the time) and the 16-RHS solve (operator and vector bytes)
    work = survey_work(nx, ny, p, nrhs)

    def stage_ms(prefixes, recs):
        return sum(v[2] for v in recs if v[0].split("@")[0].split("[")[0].startswith(prefixes))

    leaf_ms = stage_ms(("leaf_",), stages_b)
    merge_ms = stage_ms(("merge_",), stages_b)
    solve_ms_p = stage_ms(("solve_",), stages_s)
    stage_roofline = {
        "leaf": {"algorithmic_flops": work["F_leaf"], "per_leaf": work["F_leaf_per_leaf"],
                 "ms": round(leaf_ms, 3),
                 "achieved_tflops": round(work["F_leaf"] / (leaf_ms * 1e-3) / 1e12, 3),
                 "peak_tflops": 78.6,
                 "frac": round(work["F_leaf"] / (leaf_ms * 1e-3) / 78.6e12, 4),
                 # what the kernels execute: the real interior inverse (Gauss-Jordan,
                 # 2 n_i^3 per leaf on the Dirichlet route) and the complex products
                 "executed_interior_inverse_flops": 2 * (p - 2) ** 6 * nx * ny},
        "merge": {"algorithmic_flops": work["F_merge"], "ms": round(merge_ms, 3),
                  "achieved_tflops": round(work["F_merge"] / (merge_ms * 1e-3) / 1e12, 3),
                  "peak_tflops": 78.6,
                  "frac": round(work["F_merge"] / (merge_ms * 1e-3) / 78.6e12, 4)},
        "solve": {"algorithmic_bytes": work["solve_bytes"], "ms": round(solve_ms_p, 3),
                  "achieved_gbs": round(work["solve_bytes"] / (solve_ms_p * 1e-3) / 1e9, 1),
                  "peak_gbs": 8000.0,
                  "frac": round(work["solve_bytes"] / (solve_ms_p * 1e-3) / 8e12, 4)},
    }

    out = {
        "metric": METRIC,
        "value": round(dof / (ms_per_step * 1e-3), 1),
        "unit": "DOF/s (build + one 16-RHS solve per step)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128", "data": "synthetic",
        "config": {"workload": "HPS 64x64 leaves, p=16, kappa=eta=100, Gaussian-bump c, "
                               "complex128, 16 manufactured RHS per solve",
                   "leaves": nx * ny, "p": p, "dof": dof, "nrhs": nrhs},
        "build_ms": round(float(np.median(build_ms)), 3),
        "build_dof_per_s": round(dof / (np.median(build_ms) * 1e-3), 1),
        "solve_ms": round(float(np.median(solve_ms)), 3),
        "rhs_solves_per_s": round(nrhs / (np.median(lat) * 1e-3), 1),
        "solve_latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                             "p99": round(float(np.percentile(lat, 99)), 3),
                             "calls": int(len(lat)), "nrhs_per_call": nrhs},
        "rel_l2_vs_exact": err,
        "e_inf_vs_exact": einf,
        "autotune": {"gemm_shapes_tuned": H.autotune_entries(),
                     "tuning_build_s": None if tune_s is None else round(tune_s, 3)},
        "roofline": roofline,
        "stage_roofline": stage_roofline,
        "stages_ms": {k: round(v[1], 3) for k, v in groups.items()},
    }
    if not args.no_batch:
        log("batch leg")
        out["batch_256_problems"] = batch_leg(H, torch, dev, stream)
    if not args.no_serve:
        log("serving leg")
        torch.cuda.empty_cache()
        out["serving"] = serve_leg(H, torch, dev, n_requests=args.serve_requests,
                                   new_build_every=args.serve_new_every,
                                   reserve_gb=args.serve_reserve_gb)
    if not args.no_mixed:
        log("precision leg (128 x 128 leaves)")
        torch.cuda.empty_cache()
        out["precision_128x128"] = precision_leg(H, torch, dev, stream)
    if not args.no_mixed:
        out["mixed_precision"] = mixed_leg(H, torch, dom, p, kappa, c_d, s_d, t_d, u_d, exact,
                                           stream, out)
    if not args.no_cpu_baseline:
        cx, cy = (int(v) for v in args.cpu_leaves.lower().split("x"))
        log("cpu baseline (oracle) on %dx%d leaves" % (cx, cy))
        out["cpu_baseline"] = cpu_baseline(cx, cy, p, kappa, nrhs, 0)
        # the same oracle with its BLAS held to one thread, on a quarter of that sample
        try:
            from threadpoolctl import threadpool_limits
            with threadpool_limits(limits=1, user_api="blas"):
                one = cpu_baseline(max(1, cx // 2), max(1, cy // 2), p, kappa, nrhs, 0)
            out["cpu_baseline"]["single_thread"] = {k: one[k] for k in
                                                    ("value", "unit", "cores", "seconds",
                                                     "rel_l2_vs_exact", "sample")}
        except Exception as e:  # the main figure stands without it
            out["cpu_baseline"]["single_thread"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
