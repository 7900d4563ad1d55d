#!/usr/bin/env python3
"""Benchmark: exact angular pair counting (DD + DR + RR) and Landy-Szalay
w(theta) on one MI355X.

Workload: 1,000,000 clustered data points (50,000 Neyman-Scott parents x 20,
sigma 0.05 deg) and 1,000,000 area-uniform randoms on a 100 x 100 deg patch,
40 log bins 0.01-20 deg (synthetic stand-in for the paper's galaxy catalogue).
A step = one batched launch counting DD, DR and RR (1,999,999,000,000 pairs)
from float64 RA/Dec already resident in device memory, plus w(theta).

--workload aperture times the paper's second workload instead (Sec. 3):
aperture-mass and SNR maps of 10^6 synthetic galaxies at 35 per square
arcmin on a 2048 x 2048 grid with a 32 arcmin NFW filter, plus the other
grid sizes and filter radii of the paper's Table 2.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3   # MI355X: 256 CU x 4 SIMD x 16 lanes x 2 (packed) x 2 (FMA) x 2.4 GHz
PEAK_FP64_VECTOR_TFLOPS = 78.6    # MI355X binary64 vector rate (the binary64 kernel's own peak)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def work_per_pair(n_bins: int) -> int:
    """Algorithmic operations per pair: 8 flops for |a-b|^2 (3 sub, 3 mul,
    2 add) plus ceil(log2(B+2)) comparisons to place it among B+1 edges."""
    return 8 + math.ceil(math.log2(n_bins + 2))


def work_per_pair_method(n_bins: int, m: int) -> int:
    """Operations a pair needs on the path that binned it: 8 flops for the
    chord, plus ceil(log2(m+1)) comparisons when the prune pass left only m
    edges inside its chord interval (m + 1 possible rows), or
    ceil(log2(B+2)) through the cell table (m = 0: any of the B + 2 rows)."""
    return 8 + (math.ceil(math.log2(m + 1)) if m > 0 else math.ceil(math.log2(n_bins + 2)))


def cpu_model() -> str:
    """The host CPU's model name (lscpu's "Model name")."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def code_fingerprint(paths) -> str:
    """SHA-256 of the code of one source file, or of several in order (a
    kernel and the local headers its device code uses): comments removed and
    whitespace collapsed, so that editing a comment does not retire a profile
    record."""
    import hashlib
    import re
    parts = []
    for path in ([paths] if isinstance(paths, str) else paths):
        with open(path) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        parts.append(" ".join(text.split()))
    return hashlib.sha256("\n".join(parts).encode()).hexdigest()


# the sources whose code a traffic record was taken on, per kernel
K_COUNT_SOURCES = ("pc_kernels.hip", "pc_internal.hpp", "pc_math.h")
K_AP_MAP_SOURCES = ("pc_aperture.hip",)


def recorded_traffic(record: str, sources):
    """HBM bytes per launch from a committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    record, if it was taken on the kernel code as it is now; else None."""
    rec = os.path.join(ROOT, "profiles", record)
    srcs = [os.path.join(ROOT, "paper_1208_3658_amd", "csrc", x) for x in sources]
    if not os.path.exists(rec):
        return None
    with open(rec) as f:
        r = json.load(f)
    return r["traffic_bytes_per_launch"] if r.get("kernel_code_sha256") == code_fingerprint(srcs) else None


# Aperture mass (Sec. 3): algorithmic flops per galaxy-point pair inside the
# aperture, each elementary function counted as one operation: separation 5
# (2 sub, 2 mul, 1 add), cut 1, x = sqrt(d2)/theta 2, Eq. 4 13 (two
# exponentials with their arguments 6, 1 + a + b 2, reciprocal 1,
# tanh(u)/u with u = x/0.15 3, product 1), tangential ellipticity 8
# (cos 2phi 2, sin 2phi 3, e1 c + e2 s 3), sums 5 (Q eps_t and its add 2,
# Q^2 |eps|^2 and its add 3).
AP_FLOPS_PER_PAIR = 34
AP_GRIDS = (512, 1024, 2048)
AP_THETAS = (2.0, 4.0, 8.0, 16.0, 32.0)
# Table 2 of the paper: seconds per map on a Tesla M2070 (data transfer
# included) and on one CPU core; context only (other hardware).
AP_PAPER_GPU_S = {512: (11, 12, 15, 23, 45), 1024: (38, 41, 50, 78, 162), 2048: (143, 156, 190, 297, 627)}
AP_PAPER_CPU_S = {512: (558, 781, 1478, 4108, 12794), 1024: (2105, 2627, 5204, 15311, 48474),
                  2048: (8855, 11941, 22546, 61406, 189861)}


def aperture_main(args):
    import numpy as np
    import torch
    import synth
    import paper_1208_3658_amd as pc

    torch.cuda.set_device(0)
    log("generating the shear catalogue (10^6 galaxies)")
    cat, side = synth.config_aperture()
    dcat = tuple(torch.from_numpy(a).cuda() for a in cat)
    stream = torch.cuda.current_stream()
    outs = {}

    def run(grid_n, theta):
        m = grid_n * grid_n
        if grid_n not in outs:
            outs[grid_n] = {"map": torch.empty(m, dtype=torch.float64, device="cuda"),
                            "snr": torch.empty(m, dtype=torch.float64, device="cuda"),
                            "n_in": torch.empty(m, dtype=torch.int32, device="cuda")}
        pc.pc_aperture_mass(dcat, synth.field_grid(side, grid_n), theta, synth.PAPER_DENSITY, out=outs[grid_n],
                            stream=stream)
        return pc.pc_debug_last_aperture()

    G, TH = 2048, 32.0
    pc.pc_debug_set_timing(True)
    for k in range(args.warmup):
        run(G, TH)
        log(f"warmup {k + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    kern = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        info = run(G, TH)
        kern.append(info["kernel_ms"])
        log(f"step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pairs = info["pairs_in"]
    kern_s = float(np.mean(kern)) / 1e3
    achieved = pairs * AP_FLOPS_PER_PAIR / kern_s / 1e12
    table = []
    for gn in (AP_GRIDS if not args.no_table else ()):
        for ti, th in enumerate(AP_THETAS):
            run(gn, th)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            inf = run(gn, th)
            torch.cuda.synchronize()
            t1 = time.perf_counter() - t1
            table.append({"grid": gn, "theta_arcmin": th, "ms": t1 * 1e3, "kernel_ms": inf["kernel_ms"],
                          "pairs_in": inf["pairs_in"], "pairs_tested": inf["pairs_tested"],
                          "roofline_frac": inf["pairs_in"] * AP_FLOPS_PER_PAIR / (inf["kernel_ms"] / 1e3) / 1e12
                          / PEAK_FP32_VECTOR_TFLOPS,
                          "paper_m2070_s": AP_PAPER_GPU_S[gn][ti], "paper_cpu_core_s": AP_PAPER_CPU_S[gn][ti]})
            log(f"grid {gn}^2 theta {th}': {t1 * 1e3:.2f} ms (kernel {inf['kernel_ms']:.2f} ms)")
    pc.pc_debug_set_timing(False)
    out = {
        "metric": "aperture-mass map: galaxy-point pairs inside the filter radius per second",
        "value": pairs * args.steps / dt / 1e9, "unit": "Gpairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "shear_1M_35_per_arcmin2_grid2048_theta32arcmin", "galaxies": int(cat[0].size),
                   "field_arcmin": side, "grid": [G, G], "theta_max_arcmin": TH, "filter": "NFW (Eq. 4)",
                   "pairs_in_aperture": pairs},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
                     "traffic": recorded_traffic("k_ap_map_shear1M_grid2048_theta32_traffic.json", K_AP_MAP_SOURCES),
                     "kernel_ms": kern_s * 1e3,
                     "work_per_pair": AP_FLOPS_PER_PAIR, "pairs_tested": info["pairs_tested"],
                     "cell_side_arcmin": info["cell_side"]},
    }
    if table:
        out["table"] = table
    if not args.no_cpu_baseline:
        import oracle
        log("cpu baseline (oracle)")
        g = synth.field_grid(side, G)

        def sample(target):
            rng = np.random.default_rng(18)
            npts = 8
            while True:
                pick = rng.integers(0, G * G, npts)
                t = time.perf_counter()
                r = oracle.aperture_points(cat, g[0] + (pick % G) * g[2], g[1] + (pick // G) * g[3], TH,
                                           synth.PAPER_DENSITY)
                spent = time.perf_counter() - t
                pin = int(r["n_in"].sum())
                if spent >= 0.6 * target or npts >= 65536:
                    return npts, pin, spent
                npts = max(npts + 1, min(65536, int(npts * target / max(spent, 1e-3))))

        cores = oracle.num_threads()
        npts, pin, spent = sample(args.cpu_seconds)
        out["cpu_baseline"] = {"value": pin / spent / 1e9, "unit": "Gpairs/s", "cores": cores,
                               "kind": "oracle", "cpu_model": cpu_model(),
                               "sample": f"{npts} seeded points of the {G}^2 x {TH:g}' map, each against all "
                                         f"{cat[0].size} galaxies ({pin:.3e} pairs inside, {spent:.1f} s)"}
        if cores > 1:
            # the paper's speed-ups are against one CPU core (Sec. 4, Table 2)
            oracle.set_num_threads(1)
            try:
                n1, pin1, spent1 = sample(max(1.0, args.cpu_seconds / 4))
            finally:
                oracle.set_num_threads(cores)
            v1 = pin1 / spent1 / 1e9
            out["cpu_baseline"]["one_core"] = {"value": v1, "unit": "Gpairs/s", "cores": 1,
                                               "sample": f"{n1} seeded points ({pin1:.3e} pairs inside, "
                                                         f"{spent1:.1f} s)",
                                               "gpu_over_one_core": out["value"] / v1}
    print(json.dumps(out), flush=True)


def cpu_baseline(c, target_s: float):
    """The CPU oracle as it stands on a bounded row sample of the same
    workload: DD, DR and RR restricted to their first r rows."""
    import numpy as np
    import oracle
    D, R, e = c["D"], c["R"], c["edges"]
    n, nr = D[0].size, R[0].size

    def run(r):
        t = time.perf_counter()
        oracle.count(D, e, rows=(0, r))
        oracle.count(D, e, B=R, auto=False, rows=(0, r))
        oracle.count(R, e, rows=(0, r))
        dt = time.perf_counter() - t
        pairs = sum(n - 1 - i for i in range(r)) + r * nr + sum(nr - 1 - i for i in range(r))
        return pairs, dt

    def sample(target):
        r, (pairs, dt) = 16, run(16)
        for _ in range(3):                   # grow the sample until it takes ~target
            if dt >= 0.6 * target or r >= n:
                break
            r = max(r + 1, min(n, int(r * target / max(dt, 1e-3))))
            pairs, dt = run(r)
        return r, pairs, dt

    cores = oracle.num_threads()
    r, pairs, dt = sample(target_s)
    out = {"value": pairs / dt / 1e9, "unit": "Gpairs/s", "cores": cores, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": f"DD, DR and RR over the first {r} rows of the 1M workload ({pairs:.3e} pairs, {dt:.1f} s)"}
    if cores > 1:
        # the paper's speed-ups are against one CPU core (Sec. 4, Table 1)
        oracle.set_num_threads(1)
        try:
            r1, pairs1, dt1 = sample(max(1.0, target_s / 4))
        finally:
            oracle.set_num_threads(cores)
        out["one_core"] = {"value": pairs1 / dt1 / 1e9, "unit": "Gpairs/s", "cores": 1,
                           "sample": f"first {r1} rows of DD, DR and RR ({pairs1:.3e} pairs, {dt1:.1f} s)"}
    return out


def serve_oracle_check(pc, reqs, cats, randoms, results, budget_s: float, seed: int = 77):
    """Served answers against the CPU oracle, two ways.
    * whole requests: DD and DR of the smallest requests, smallest first,
      until about half of budget_s seconds of oracle time are spent;
    * every request: its served DD, DR and RR equal one direct launch of the
      same jobs (pc_count_batch on the same catalogues and edges), and windows
      of 8 data rows of that request's DR (seeded) and DD (near the end of
      the catalogue), counted by the library (pc_count_ex row range) and by
      the oracle, agree: the oracle pins a sample of every request's counts,
      the direct launch ties them to the served answer.
    (RR of a 10^6-point pool catalogue is 5e11 pairs per edge set, minutes of
    oracle time each: RR is tied to the direct launch only; the tests pin the
    library's RR against the oracle.)"""
    import numpy as np
    import oracle
    order = sorted(range(len(reqs)), key=lambda k: (cats[k][0].size, k))
    t0 = time.perf_counter()
    checked, same, n_max, pairs = 0, True, 0, 0
    for k in order:
        if time.perf_counter() - t0 > 0.5 * budget_s:
            break
        r, cat, res = reqs[k], cats[k], results[k]
        R = randoms[r["patch"]]
        dd = oracle.count(cat, r["edges"])
        dr = oracle.count(cat, r["edges"], B=R, auto=False)
        same &= res["DD"].tolist() == dd.tolist() and res["DR"].tolist() == dr.tolist()
        checked += 1
        n_max = max(n_max, int(cat[0].size))
        pairs += int(dd.sum()) + int(dr.sum())
    whole_s = time.perf_counter() - t0
    import torch

    def dev(cat):
        return tuple(torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in cat)

    rng = np.random.default_rng(seed)
    t1 = time.perf_counter()
    r_dev = [dev(R) for R in randoms]                       # the pool catalogues, once
    r_xyz = [oracle.unit_vectors(*R) for R in randoms]

    def oracle_rows(cat, e, p, dr_rows, dd_rows):
        # DR: data rows dr_rows against all randoms; DD: pairs i < j with i
        # in dd_rows, from the catalogue's tail (the oracle converts only that)
        c2 = oracle.chord2_edges(e)
        (a, b), (t0_, t1_) = dr_rows, dd_rows
        o_dr = oracle.count_xyz(oracle.unit_vectors(cat[0][a:b], cat[1][a:b]), c2, r_xyz[p], auto=False)
        o_dd = oracle.count_xyz(oracle.unit_vectors(cat[0][t0_:], cat[1][t0_:]), c2, rows=(0, t1_ - t0_))
        return o_dd, o_dr

    from concurrent.futures import ThreadPoolExecutor
    direct_same, rows_same, row_pairs = True, True, 0
    pending = []
    with ThreadPoolExecutor(max_workers=8) as pool:
        for k, (r, cat, res) in enumerate(zip(reqs, cats, results)):
            p, e = r["patch"], r["edges"]
            d_cat = dev(cat)
            dd, dr, rr = pc.pc_count_batch([{"A": d_cat, "edges": e},
                                            {"A": d_cat, "B": r_dev[p], "edges": e, "auto": False},
                                            {"A": r_dev[p], "edges": e}])
            direct_same &= (res["DD"].tolist() == dd.tolist() and res["DR"].tolist() == dr.tolist()
                            and res["RR"].tolist() == rr.tolist())
            # a seeded window of W data rows for DR; for DD the W rows that
            # start 2048 rows before the catalogue's end
            n, W = int(cat[0].size), 8
            a = int(rng.integers(0, max(n - W, 0) + 1))
            dr_rows = (a, min(a + W, n))
            t0_ = max(n - 2048 - W, 0)
            dd_rows = (t0_, min(t0_ + W, n))
            g_dr = pc.pc_count_ex(d_cat, e, B=r_dev[p], auto=False, rows=dr_rows)
            g_dd = pc.pc_count_ex(d_cat, e, rows=dd_rows)
            pending.append((g_dd, g_dr, pool.submit(oracle_rows, cat, e, p, dr_rows, dd_rows)))
        for g_dd, g_dr, fut in pending:
            o_dd, o_dr = fut.result()
            rows_same &= g_dd.tolist() == o_dd.tolist() and g_dr.tolist() == o_dr.tolist()
            row_pairs += int(o_dd.sum()) + int(o_dr.sum())
    return {"requests": checked, "of": len(reqs), "n_max": n_max, "pairs": pairs, "identical_dd_dr": bool(same),
            "oracle_s": whole_s, "threads": oracle.num_threads(),
            "sample": "the smallest requests (whole DD and DR) within half the oracle time budget",
            "every_request": {"requests": len(reqs), "served_equal_direct_launch_dd_dr_rr": bool(direct_same),
                              "row_window": 8, "row_window_pairs": row_pairs,
                              "rows_identical_to_oracle_dd_dr": bool(rows_same),
                              "seconds": time.perf_counter() - t1}}


def serve_run(pc, n_req: int, seed_config: int = 5, loads=(0.7,), fp64_compare: bool = True, server_cfg=None,
              oracle_seconds: float = 0.0):
    """Stream of w(theta) requests (config: N log-uniform 1e3..2e6, clustered
    on one of 4 pool patches of side 5-50 deg, 10-50 log bins).  The server's
    capacity on this stream is measured first (every request submitted at
    once); then Poisson arrivals at each load (fraction of that capacity) give
    the latencies of the mixed-precision batched server; at 0.7 the same
    arrivals are also replayed against a binary64 server that runs one
    request per launch."""
    import numpy as np
    import synth
    from synth.catalogs import pool_random, request_catalog
    patches, reqs = synth.serve_stream(n_req, rate_hz=1.0, n_patches=4, seed_config=seed_config)
    cats = [request_catalog(patches, r, seed_config) for r in reqs]
    randoms = [pool_random(patches, p, seed_config) for p in range(len(patches))]

    def run(arrivals, cfg):
        srv = pc.Server(cfg)
        for p, R in enumerate(randoms):
            srv.set_random(p, R)
        t0 = time.perf_counter()
        ids = []
        for k, (r, cat) in enumerate(zip(reqs, cats)):
            wait = arrivals[k] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            ids.append(srv.submit(cat, r["patch"], r["edges"]))
        srv.drain()
        wall = time.perf_counter() - t0
        res = [srv.poll(j) for j in ids]
        st = srv.stats()
        srv.close()
        lat_raw = np.array([x["latency_s"] for x in res])
        lat = np.sort(lat_raw)
        # where the tail lives: latencies of the requests grouped by their
        # DD + DR pairs (quantiles of request size)
        size = np.array([r["n"] * (r["n"] - 1) / 2 + r["n"] * randoms[r["patch"]][0].size for r in reqs])
        by_size, order = [], np.argsort(size, kind="stable")
        for q0, q1 in ((0.0, 0.5), (0.5, 0.9), (0.9, 0.99), (0.99, 1.0)):
            sel = order[int(round(q0 * len(order))):int(round(q1 * len(order)))]
            if sel.size:
                ls = lat_raw[sel]
                by_size.append({"size_quantiles": [q0, q1], "requests": int(sel.size),
                                "max_pairs": float(size[sel].max()), "p50_s": float(np.percentile(ls, 50)),
                                "p99_s": float(np.percentile(ls, 99)), "max_s": float(ls.max())})
        return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "gpairs_s": st["pairs"] / wall / 1e9, "wall_s": wall, "batches": st["batches"],
                "rr_cached": st["rr_cached"], "parts_requeued": st.get("parts_requeued", 0),
                "slice_pairs": st.get("slice_pairs"), "latency_by_size": by_size}, res

    mixed_cfg = {"streams": 2, "max_inflight": 64, **(server_cfg or {})}
    closed, _ = run(np.zeros(n_req), mixed_cfg)
    capacity = n_req / closed["wall_s"]
    unit_gaps = np.random.Generator(np.random.PCG64(1000 * seed_config + 4)).exponential(1.0, n_req)
    log(f"serve: capacity {capacity:.2f} requests/s on this stream")
    out = {"requests": n_req, "capacity_rps": capacity}
    for load in loads:
        rate = load * capacity
        arrivals = np.cumsum(unit_gaps / rate)
        mixed, res_m = run(arrivals, mixed_cfg)
        log(f"serve at {load:.1f} x capacity ({rate:.2f}/s): p50 {mixed['p50_s']:.3f} s, p99 {mixed['p99_s']:.3f} s")
        if abs(load - 0.7) < 1e-9:
            out.update({"rate_hz": rate, **mixed})
            if oracle_seconds > 0:
                out["oracle_check"] = serve_oracle_check(pc, reqs, cats, randoms, res_m, oracle_seconds)
            if fp64_compare:
                single64, res_f = run(arrivals, {"streams": 1, "max_inflight": 64, "max_batch_pairs": 1,
                                                 "mode": pc.PC_FP64_PLAIN})
                out["fp64_one_request_per_launch"] = single64
                out["identical_counts"] = all(a[k].tolist() == b[k].tolist() for a, b in zip(res_m, res_f)
                                              for k in ("DD", "DR", "RR"))
        else:
            out.setdefault("load_sweep", []).append({"load": load, "rate_hz": rate, **mixed})
    return out


def build_workload(name, torch, pc):
    """Jobs of one step, the (DD, DR, RR) job indices of each w(theta), total
    pairs and bin count."""
    import synth

    def dev(cat):
        return tuple(torch.from_numpy(x).cuda() for x in cat)

    if name in ("1m", "large", "paper"):
        c = {"1m": synth.config_1m, "large": synth.config_large}.get(name, lambda: synth.paper_shape(1_000_000))()
        D, R, e = dev(c["D"]), dev(c["R"]), c["edges"]
        nD, nR = D[0].numel(), R[0].numel()
        c["describe"] = {"n_data": nD, "n_random": nR, "theta_deg": [float(e[0]), float(e[-1])]}
        if name == "paper":
            jobs = [{"A": D, "B": R, "edges": e, "auto": False}]
            return c, jobs, [], nD * nR, e.size - 1
        jobs = [{"A": D, "edges": e}, {"A": D, "B": R, "edges": e, "auto": False}, {"A": R, "edges": e}]
        pairs = nD * (nD - 1) // 2 + nD * nR + nR * (nR - 1) // 2
        return c, jobs, [(0, 1, 2, nD, nR)], pairs, e.size - 1
    c = synth.config_batched()
    R, e = dev(c["R"]), c["edges"]
    nR = R[0].numel()
    jobs, est, pairs = [], [], 0
    rr = 2 * len(c["mocks"])
    for m in c["mocks"]:
        M = dev(m)
        n = M[0].numel()
        est.append((len(jobs), len(jobs) + 1, rr, n, nR))
        jobs += [{"A": M, "edges": e}, {"A": M, "B": R, "edges": e, "auto": False}]
        pairs += n * (n - 1) // 2 + n * nR
    jobs.append({"A": R, "edges": e})
    pairs += nR * (nR - 1) // 2
    c["describe"] = {"n_mocks": len(c["mocks"]), "n_data_total": sum(m[0].size for m in c["mocks"]),
                     "n_random": nR, "theta_deg": [float(e[0]), float(e[-1])]}
    c.pop("mocks")
    return c, jobs, est, pairs, e.size - 1


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--matrix-cores", action="store_true",
                    help="time the mixed mode with the matrix-core chord path (PC_MATRIX_CORES) "
                         "as the main step")
    ap.add_argument("--no-matrix-compare", action="store_true",
                    help="skip the extra step with the matrix-core chord path")
    ap.add_argument("--no-autotune", action="store_true",
                    help="run the default launch parameters instead of tuning them on the first step")
    ap.add_argument("--tune-cache", default=None, metavar="PATH",
                    help="tuned launch parameters: use the entries in PATH if it exists (no tuning run), "
                         "else tune and write them there")
    ap.add_argument("--workload", choices=["1m", "batched", "large", "paper", "aperture"], default="1m",
                    help="1m: 1M clustered + 1M random (default); batched: 256 mocks x shared 1M random; "
                         "large: 4M + 8M full sky; paper: DR of 1M + 1M uniform, 254 log bins; "
                         "aperture: aperture-mass maps of 1M galaxies (Sec. 3)")
    ap.add_argument("--no-table", action="store_true",
                    help="aperture workload: time only the 2048^2 x 32 arcmin map, not the grid/radius table")
    ap.add_argument("--per-job-launches", action="store_true",
                    help="also time the same jobs with one launch each")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-host-compare", action="store_true",
                    help="skip the extra step from host-memory catalogues (upload included)")
    ap.add_argument("--no-prune-compare", action="store_true",
                    help="skip the extra step that visits every pair")
    ap.add_argument("--serve-requests", type=int, default=300)
    ap.add_argument("--serve-oracle-seconds", type=float, default=15.0,
                    help="CPU oracle time spent checking served answers (smallest requests first); 0: none")
    ap.add_argument("--serve-config", default="",
                    help="JSON object of pc_server_create keys overriding the mixed server's (e.g. streams)")
    ap.add_argument("--serve-loads", default="0.7", metavar="F,F,...",
                    help="Poisson arrival rates as fractions of the measured capacity (0.7 is always reported)")
    ap.add_argument("--no-serve-fp64-compare", action="store_true",
                    help="skip the replay against one binary64 launch per request")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (for scaling HBM counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding is not built: "
              "tile-pair ranges would split across GPUs with one all-reduce of the histograms",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "aperture":
        aperture_main(args)
        return

    import numpy as np
    import torch
    import synth
    import paper_1208_3658_amd as pc

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        log(f"copied {args.copy_calibration} MiB")
        return
    log(f"generating workload {args.workload}")
    c, jobs, est, pairs, n_bins = build_workload(args.workload, torch, pc)
    mode = pc.PC_MIXED if args.mode == "mixed" else pc.PC_FP64_PLAIN
    if args.matrix_cores and mode == pc.PC_MIXED:
        mode |= pc.PC_MATRIX_CORES
    stream = torch.cuda.current_stream()

    def step(m):
        counts = pc.pc_count_batch(jobs, mode=m, stream=stream)
        ws = [pc.pc_wtheta(counts[a][1:-1], counts[b][1:-1], counts[r][1:-1], nd, nr) for a, b, r, nd, nr in est]
        return counts, ws

    tuned = None
    if not args.no_autotune and not (mode & pc.PC_MATRIX_CORES):
        if args.tune_cache and os.path.exists(args.tune_cache):
            pc.pc_autotune_load(args.tune_cache)
            with open(args.tune_cache) as f:
                tuned = {"loaded_from": args.tune_cache, "entries": [json.loads(l) for l in f if l.strip()]}
        else:
            # choose the launch parameters on this batch (untimed; counts
            # checked equal across all candidates), then run the steps with them
            _, tuned = pc.pc_autotune(jobs, mode=mode, cache_path=args.tune_cache, stream=stream)
        mode |= pc.PC_TUNED
        log(f"autotune: {tuned}")
    pc.pc_debug_set_timing(True)
    for k in range(args.warmup):
        step(mode)
        log(f"warmup {k + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    kern = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        counts, ws = step(mode)
        kern.append(pc.pc_debug_last_launch()["kernel_ms"])
        log(f"step {k + 1}/{args.steps} done")
    prn = pc.pc_debug_last_pruning()
    paths = pc.pc_debug_last_paths()
    rechecked = pc.pc_debug_last_rechecks()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launch = pc.pc_debug_last_launch()
    assert sum(int(x.sum()) for x in counts) == pairs
    value = pairs * args.steps / dt / 1e9
    kern_s = float(np.mean(kern)) / 1e3
    W = work_per_pair(n_bins)
    # the pair kernel's own rate: the pairs it visits one by one (tile pairs
    # binned whole by the bounding-sphere test never reach it)
    achieved = prn["pairs_computed"] * W / kern_s / 1e12
    fp64_run = (mode & 0xFF) == pc.PC_FP64_PLAIN
    peak = PEAK_FP64_VECTOR_TFLOPS if fp64_run else PEAK_FP32_VECTOR_TFLOPS
    # the same rate counting, per pair, only the comparisons its path needs
    # (few-edge pairs compare with the m <= 3 edges left in their interval)
    by = paths["by_edges"]
    assert sum(by) == prn["pairs_computed"], (by, prn["pairs_computed"])
    work_method = sum(by[m] * work_per_pair_method(n_bins, m) for m in range(4))
    achieved_method = work_method / kern_s / 1e12
    out = {
        "metric": "Gpairs/s binned (DD+DR+RR) at N=1M; p50/p99 latency of served w(theta) jobs",
        "value": value, "unit": "Gpairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if fp64_run else "f32+f64", "data": "synthetic",
        "config": {"workload": c["name"], **c["describe"], "bins": n_bins, "jobs_per_launch": len(jobs),
                   "pairs_per_step": pairs,
                   "mode": args.mode + ("+matrix_cores" if mode & pc.PC_MATRIX_CORES else "")
                   + ("+tuned" if mode & pc.PC_TUNED else "")},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": recorded_traffic("k_count_mixed_1M_traffic.json", K_COUNT_SOURCES)
                     if args.workload == "1m" and args.mode == "mixed" else None,
                     "frac_method": achieved_method / peak, "achieved_method": achieved_method,
                     "work_per_pair_method": work_method / max(prn["pairs_computed"], 1),
                     "pairs_by_path": {"cell_table": by[0], "one_edge": by[1], "two_edges": by[2],
                                       "three_edges": by[3], "gram_form": paths["gram"],
                                       "difference_form": prn["pairs_computed"] - paths["gram"] - paths["mfma"],
                                       "matrix_cores": paths["mfma"]},
                     "kernel_ms": kern_s * 1e3, "work_per_pair": W, "grid": launch["grid"],
                     "lds_bytes": launch["lds_bytes"], "items": launch["items"],
                     "pairs_computed": prn["pairs_computed"], "survivor_items": prn["survivors"],
                     "few_edge_items": prn["few_items"], "gram_form_items": prn["gram_items"],
                     "matrix_core_items": prn["mfma_items"],
                     "computed_gpairs_s": prn["pairs_computed"] / kern_s / 1e9,
                     # the chord alone (8 flops per pair), for comparison with the full count W
                     "chord_only_frac": prn["pairs_computed"] * 8 / kern_s / 1e12 / peak},
        "pairs_binned_whole": pairs - prn["pairs_computed"],
        # pairs whose binary32 chord fell in an edge's guard band (re-checked in binary64)
        "rechecks": {"pairs": rechecked, "of_computed": rechecked / max(prn["pairs_computed"], 1),
                     "of_all": rechecked / pairs},
        "launch_tuning": tuned,
    }
    pc.pc_debug_set_timing(False)
    if args.no_prune_compare is False:
        # the same step visiting every pair (no whole-tile-pair binning)
        pc.pc_debug_set_timing(True)
        t1 = time.perf_counter()
        counts3, _ = step(mode | pc.PC_NO_PRUNE)
        torch.cuda.synchronize()
        t1 = time.perf_counter() - t1
        k3 = pc.pc_debug_last_launch()["kernel_ms"] / 1e3
        pc.pc_debug_set_timing(False)
        out["every_pair"] = {"value": pairs / t1 / 1e9, "ms_per_step": t1 * 1e3, "kernel_ms": k3 * 1e3,
                             "roofline_frac": pairs * W / k3 / 1e12 / PEAK_FP32_VECTOR_TFLOPS,
                             "identical_counts": all(a.tolist() == b.tolist() for a, b in zip(counts, counts3))}
        log(f"every-pair step {t1 * 1e3:.1f} ms")
    base_mode = mode & ~(pc.PC_MATRIX_CORES | pc.PC_TUNED)
    main_mc = bool(tuned.get("matrix_cores", 0)) if tuned else bool(mode & pc.PC_MATRIX_CORES)
    if not args.no_matrix_compare and base_mode == pc.PC_MIXED:
        # the same step with the other choice of chord path (default launch
        # parameters otherwise)
        other = pc.PC_MIXED | (0 if main_mc else pc.PC_MATRIX_CORES)
        step(other)
        pc.pc_debug_set_timing(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        counts4, _ = step(other)
        torch.cuda.synchronize()
        t4 = time.perf_counter() - t1
        k4 = pc.pc_debug_last_launch()["kernel_ms"]
        pc.pc_debug_set_timing(False)
        key = "matrix_cores" if other & pc.PC_MATRIX_CORES else "vector_only"
        out[key] = {"value": pairs / t4 / 1e9, "ms_per_step": t4 * 1e3, "kernel_ms": k4,
                    "matrix_core_items": pc.pc_debug_last_pruning()["mfma_items"],
                    "identical_counts": all(a.tolist() == b.tolist() for a, b in zip(counts, counts4))}
        log(f"{key} step {t4 * 1e3:.1f} ms (kernel {k4:.1f} ms)")
    if not args.no_fp64_compare and base_mode == pc.PC_MIXED:
        step(pc.PC_FP64_PLAIN)
        torch.cuda.synchronize()
        pc.pc_debug_set_timing(True)
        t1 = time.perf_counter()
        counts2, _ = step(pc.PC_FP64_PLAIN)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        k64 = pc.pc_debug_last_launch()["kernel_ms"] / 1e3
        p64 = pc.pc_debug_last_pruning()["pairs_computed"]
        pc.pc_debug_set_timing(False)
        same = all(a.tolist() == b.tolist() for a, b in zip(counts, counts2))
        # the binary64 kernel against the binary64 vector peak
        out["fp64_plain"] = {"value": pairs / t64 / 1e9, "ms_per_step": t64 * 1e3, "kernel_ms": k64 * 1e3,
                             "pairs_computed": p64,
                             "roofline_frac": p64 * W / k64 / 1e12 / PEAK_FP64_VECTOR_TFLOPS,
                             "identical_counts": same}
        log(f"fp64 plain step {t64 * 1e3:.1f} ms, identical counts: {same}")
    if args.workload == "1m" and not args.no_host_compare:
        # the same step from catalogues in host memory: the upload (2 x 16 MB
        # of binary64 RA/Dec) is inside the timed call, as in the paper's times
        hjobs = [{"A": c["D"], "edges": c["edges"]}, {"A": c["D"], "B": c["R"], "edges": c["edges"], "auto": False},
                 {"A": c["R"], "edges": c["edges"]}]
        pc.pc_count_batch(hjobs, mode=mode, stream=stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        hcounts = pc.pc_count_batch(hjobs, mode=mode, stream=stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter() - t1
        out["host_inputs"] = {"value": pairs / t1 / 1e9, "ms_per_step": t1 * 1e3,
                              "identical_counts": all(a.tolist() == b.tolist() for a, b in zip(counts, hcounts))}
        log(f"host-input step {t1 * 1e3:.1f} ms")
    if args.per_job_launches:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        single = [pc.pc_count_batch([j], mode=mode, stream=stream)[0] for j in jobs]
        torch.cuda.synchronize()
        t1 = time.perf_counter() - t1
        out["per_job_launches"] = {"value": pairs / t1 / 1e9, "ms": t1 * 1e3, "launches": len(jobs),
                                   "identical_counts": all(a.tolist() == b.tolist() for a, b in zip(counts, single))}
        log(f"one launch per job: {t1 * 1e3:.1f} ms")
    if args.serve_requests > 0 and args.workload == "1m":
        loads = sorted({0.7, *(float(x) for x in args.serve_loads.split(",") if x.strip())})
        out["serve"] = serve_run(pc, args.serve_requests, loads=loads, fp64_compare=not args.no_serve_fp64_compare,
                                 server_cfg=json.loads(args.serve_config) if args.serve_config else None,
                                 oracle_seconds=0.0 if args.no_cpu_baseline else args.serve_oracle_seconds)
        if args.serve_config:
            out["serve"]["server_config"] = json.loads(args.serve_config)
        if "fp64_one_request_per_launch" in out["serve"]:
            log(f"serve: binary64 one per launch: p50 {out['serve']['fp64_one_request_per_launch']['p50_s']:.3f} s, "
                f"p99 {out['serve']['fp64_one_request_per_launch']['p99_s']:.3f} s")
    if not args.no_cpu_baseline and args.workload == "1m":
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(c, args.cpu_seconds)
        if "one_core" in out["cpu_baseline"]:
            one = out["cpu_baseline"]["one_core"]
            one["gpu_over_one_core"] = out["value"] / one["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
