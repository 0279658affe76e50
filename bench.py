"""Benchmark of the served ACA weak-form entry path.

Default workload (the largest single-GPU configuration): the served Laplace
single layer, P1, on the 1,049,540-triangle capped cylinder (R = 1, L = 16,
vertices jittered by +-1% of the edge, seed 0), 6-point rule, H-matrix leaf
16, eta = 1, largest admissible block 4,096, ACA tolerance 1e-5, 32 host ACA
workers.  The admissible blocks are drawn in a seeded order (seed 2) and cut
into warmup + steps segments that together cover the whole matrix once; one
step = one segment served as a stream whose blocks arrive as a Poisson
process (seed 1) at an offered load above the capacity measured on the
warm-up segments, so the timed steps measure what the device path sustains
while requests arrive continuously.  `value` = ACA entries evaluated per
second of wall time over the timed steps (host ACA in FP64, batching,
device kernels, transfers); p50/p99 = submit -> completion latency of the
ACA row/column requests of the timed steps.  The same segments with plain
FP64 entries form the FP64 leg; extra segments at 50/80/95% of capacity give
latency against load.

The roofline object is for the dominant kernel (largest summed duration):
algorithmic flops per launch / mean launch duration, the duration from the
server's HIP events around each launch on its stream (what rocprofv3's
kernel trace also reports).  `cpu_baseline` times the FP64 oracle on a
bounded seeded sample of the same ACA row/column requests, on all host
threads and on one.

Other workloads: --workload icosphere6 (Laplace single + double layer, P1,
81,920-triangle icosphere, leaf 100, H-matrix assembly per step), --dense,
--complete.

Usage: python bench.py [--gpus 1] [--steps 3] [--warmup 1]
"""
import argparse
import hashlib
import json
import math
import os
import resource
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic flops per kernel evaluation (one pair of quadrature points),
# the per-unit figures of the hot-path measurement plan: FMA = 2, add/mul = 1,
# rsq/sin/cos = 1 each.  Laplace single layer 11 (P0) / 15 (P1, three trial
# accumulators), double layer 19 / 23 (the (x-y).n_y product per pair),
# Helmholtz single layer 20 / 28, double layer 33 / 41.
FLOPS_PER_EVAL = {(0, 0): 11, (1, 0): 19, (2, 0): 20, (3, 0): 33,
                  (0, 1): 15, (1, 1): 23, (2, 1): 28, (3, 1): 41,
                  # hypersingular (P1), by the same rules: the plain pair sum of g
                  # (Laplace 11, as the P0 single layer; Helmholtz 20) plus, for
                  # Helmholtz, the basis-weighted complex sum (4)
                  (6, 1): 11, (7, 1): 24}
# What the kernels execute per evaluation after hoisting the (x-y).n_y
# product (constant over a trial triangle's points) and the basis weights
# out of the inner loop: reported beside the algorithmic rate.
FLOPS_EXECUTED = {(0, 0): 11, (1, 0): 13, (2, 0): 21, (3, 0): 27,
                  (0, 1): 12, (1, 1): 14, (2, 1): 22, (3, 1): 28,
                  (6, 1): 10, (7, 1): 29}
# MI355X FP32 vector peak, the published figure: 256 CUs x 4 SIMDs x 16 lanes
# x 2 flops (FMA) x 2 (packed two-wide FP32) x 2.4 GHz = 157.3 TFLOP/s.  The
# device code is built without packed FP32 instructions, so the rate it can
# reach is the unpacked half, 78.6 TFLOP/s, reported beside the fraction.
PEAK_FP32_VALU = 256 * 4 * 16 * 2 * 2.4e9
PEAK_FP32_PACKED = 2 * PEAK_FP32_VALU
KERNEL_NAMES = {0: "k_p0", 1: "k_p1"}
def traffic_file(workload):
    """Calibrated HBM traffic record of the dominant kernel of a workload."""
    return os.path.join(ROOT, "profiles", f"traffic_{workload}_p1.json")


def kernel_source_hash():
    with open(os.path.join(ROOT, "paper_1711_01897_amd", "csrc", "entries.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cylinder", choices=["cylinder", "icosphere6", "spheroid", "mix", "sphere3"],
                    help="cylinder: the served 1,049,540-triangle capped cylinder (default); icosphere6: H-matrix "
                         "assembly of the Laplace single and double layer on the level-6 icosphere per step; spheroid: "
                         "H-matrix of the Helmholtz single layer, P0, on the 262,186-triangle 10:1:1 spheroid, "
                         "complex64 vs complex128; mix: served Helmholtz single layer on 8 meshes x 4 wavenumbers; "
                         "sphere3: the dense P0 Laplace single layer of the level-3 icosphere, FP64")
    ap.add_argument("--workers", type=int, default=None, help="host ACA workers (cylinder and mix 32, icosphere6 12, others 10)")
    ap.add_argument("--blocks-per-worker", type=int, default=None,
                    help="ACA blocks each worker keeps in flight (cylinder 128, icosphere6 180)")
    ap.add_argument("--load", type=float, default=1.25,
                    help="cylinder: offered block arrival rate of the timed steps as a multiple of the capacity "
                         "measured on the warm-up segments")
    ap.add_argument("--sweep", default="0.5,0.8,0.95",
                    help="cylinder: offered loads of the extra latency-against-load segments ('' for none)")
    ap.add_argument("--mix-fraction", type=float, default=0.125,
                    help="mix: the seeded share of every instance's admissible blocks served (1.0: all 16.8M)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-star", action="store_true", help="--dense: skip the star-kernel comparison")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-hmatrix-fraction", type=float, default=0.02,
                    help="icosphere6: fraction of admissible blocks in the CPU-only oracle H-matrix assembly "
                         "(0: skip)")
    ap.add_argument("--dense", type=int, default=0, metavar="LEVEL",
                    help="instead of the H-matrix workload: the dense P1 matrix of the --ops operators on the "
                         "icosphere of this level, submitted to the request server in row chunks")
    ap.add_argument("--complete", type=int, default=0, metavar="LEVEL",
                    help="instead of the ACA workload: complete P0 H-matrices (dense leaves with their singular "
                         "pairs) on the icosphere of this level, FP64")
    ap.add_argument("--complete-op", default="laplace_slp",
                    choices=["laplace_slp", "laplace_dlp", "helmholtz_slp", "helmholtz_dlp", "laplace_hyps",
                             "helmholtz_hyps"],
                    help="operator of --complete (Helmholtz at 10 elements per wavelength; the hypersingular "
                         "operators with --complete-space p1)")
    ap.add_argument("--complete-space", default="p0", choices=["p0", "p1"],
                    help="space of --complete (P0 or P1; the hypersingular operators need P1)")
    ap.add_argument("--concurrent", type=int, default=0,
                    help="1: assemble the step's operators at the same time (one host thread each, the workers "
                         "split between them), as concurrent clients of the request server")
    ap.add_argument("--ops", default="laplace_slp,laplace_dlp",
                    help="operators assembled per step (comma list of laplace_slp, laplace_dlp, laplace_adlp, "
                         "laplace_hyps); the default is the stated workload")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run a plain device copy of this many bytes (counter calibration)")
    ap.add_argument("--traffic-from", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="only summarise four rocprofv3 --pmc runs (FETCH_SIZE and WRITE_SIZE of this benchmark and "
                         "of --copy-calibration) into the traffic record used by the roofline")
    ap.add_argument("--traffic-kernel", default="k_p1_f32<1, 6>",
                    help="kernel name fragment of the dominant kernel for --traffic-from")
    ap.add_argument("--traffic-copy-bytes", type=int, default=256 << 20)
    a = ap.parse_args()
    if a.workers is None:
        a.workers = {"cylinder": 32, "mix": 32, "icosphere6": 12}.get(a.workload, 10)
    if a.blocks_per_worker is None:
        a.blocks_per_worker = 128 if a.workload in ("cylinder", "mix") else 180
    return a


def copy_calibration(nbytes):
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "dispatches": 5}))


def _counter_rows(d):
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "*counter_collection.csv"))):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    if not rows:
        raise SystemExit(f"no counter_collection.csv under {d}")
    return rows


def _mean_kib(rows, counter, pick):
    """Mean counter value per dispatch of the picked kernel, the dispatch
    count and the counter's sum over all workgroups of those dispatches
    divided by their workgroups (per-workgroup mean)."""
    sel = [r for r in rows if r["Counter_Name"] == counter and pick(r["Kernel_Name"])]
    if not sel:
        raise SystemExit(f"no {counter} rows for the requested kernel")
    vals = [float(r["Counter_Value"]) for r in sel]
    wgs = [max(1, int(r["Grid_Size"]) // max(1, int(r["Workgroup_Size"]))) for r in sel]
    return sum(vals) / len(vals), len(vals), sum(vals) / sum(wgs)


def traffic_from(args):
    """HBM traffic per launch of the dominant kernel from two --pmc runs
    (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by what the same
    counter reads for a device copy of known size."""
    fdir, wdir, cfdir, cwdir = args.traffic_from
    frag = args.traffic_kernel
    is_dom = lambda name: frag in name
    is_copy = lambda name: "copyBuffer" in name
    fetch, nf, fetch_wg = _mean_kib(_counter_rows(fdir), "FETCH_SIZE", is_dom)
    write, nw, write_wg = _mean_kib(_counter_rows(wdir), "WRITE_SIZE", is_dom)
    # the copy reads and writes args.traffic_copy_bytes; take its largest dispatch
    cf = max(float(r["Counter_Value"]) for r in _counter_rows(cfdir)
             if r["Counter_Name"] == "FETCH_SIZE" and is_copy(r["Kernel_Name"]))
    cw = max(float(r["Counter_Value"]) for r in _counter_rows(cwdir)
             if r["Counter_Name"] == "WRITE_SIZE" and is_copy(r["Kernel_Name"]))
    kib = args.traffic_copy_bytes / 1024.0
    f_fetch, f_write = kib / cf, kib / cw
    rec = {"kernel": frag, "kernel_source_hash": kernel_source_hash(),
           "fetch_kib_per_dispatch": fetch, "write_kib_per_dispatch": write, "dispatches": [nf, nw],
           "copy_bytes": args.traffic_copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
           "fetch_factor": f_fetch, "write_factor": f_write,
           "bytes_per_launch": (fetch * f_fetch + write * f_write) * 1024.0,
           # per workgroup: launch sizes differ between the counter runs and
           # the timed run, so the roofline scales this by its own launches
           "bytes_per_workgroup": (fetch_wg * f_fetch + write_wg * f_write) * 1024.0}
    with open(traffic_file(args.workload), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


OP_NAMES = {"laplace_slp": 0, "laplace_dlp": 1, "laplace_adlp": 4, "laplace_hyps": 6}
OP_LABEL = {0: "single", 1: "double", 4: "adjoint double", 6: "hypersingular"}


def step_ops(args):
    return [OP_NAMES[o] for o in args.ops.split(",")]


def workload_name(args):
    kinds = "single+double layer" if step_ops(args) == [0, 1] else \
        " + ".join(OP_LABEL[o] for o in step_ops(args)) + " operator"
    return (f"icosphere level 6 (81920 triangles, 40962 vertices), Laplace {kinds}, P1, 6-point rule, H-matrix leaf "
            "100, eta 1.0, ACA tol 1e-5, every ACA row/column on the GPU through the request server, FP32 compensated "
            "entries")


def assemble_step(bem, mesh, prec, args):
    out = {"entries": 0, "requests": 0, "rank_sum": 0, "rank_max": 0, "blocks": 0, "phases": {}}
    ops = step_ops(args)
    if args.concurrent and len(ops) > 1:
        import threading
        workers = max(1, args.workers // len(ops))
        done = {}

        def one(op):
            done[op] = bem.hmat_assemble(mesh, op, bem.P1, 0.0, leaf_size=100, eta=1.0, aca_tol=1e-5, max_rank=200,
                                         n_workers=workers, blocks_per_worker=args.blocks_per_worker, prec=prec,
                                         dense_mode=0)
        th = [threading.Thread(target=one, args=(op,)) for op in ops]
        for t in th:
            t.start()
        for t in th:
            t.join()
        results = [done[op] for op in ops]
    else:
        results = (bem.hmat_assemble(mesh, op, bem.P1, 0.0, leaf_size=100, eta=1.0, aca_tol=1e-5, max_rank=200,
                                     n_workers=args.workers, blocks_per_worker=args.blocks_per_worker, prec=prec,
                                     dense_mode=0) for op in ops)
    for H in results:
        st = H.stats()
        out["entries"] += st["aca_entries"]
        out["requests"] += st["aca_requests"]
        out["rank_sum"] += st["rank_sum"]
        out["rank_max"] = max(out["rank_max"], st["rank_max"])
        out["blocks"] += st["admissible_blocks"]
        for key in ("seconds", "partition_seconds", "setup_seconds", "aca_seconds", "worker_busy_seconds"):
            out["phases"][key] = out["phases"].get(key, 0.0) + st[key]
        H.destroy()
    return out


def timed(bem, mesh, prec, steps, warmup, args):
    import torch
    for _ in range(warmup):
        assemble_step(bem, mesh, prec, args)
    bem.server_stats(reset=True)
    bem.server_kernel_stats(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot = {"entries": 0, "requests": 0, "rank_sum": 0, "rank_max": 0, "blocks": 0, "phases": {}, "step_seconds": []}
    for _ in range(steps):
        ts = time.perf_counter()
        s = assemble_step(bem, mesh, prec, args)
        tot["step_seconds"].append(time.perf_counter() - ts)
        for k in ("entries", "requests", "rank_sum", "blocks"):
            tot[k] += s[k]
        for k, v in s["phases"].items():
            tot["phases"][k] = tot["phases"].get(k, 0.0) + v / steps
        tot["rank_max"] = max(tot["rank_max"], s["rank_max"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, tot, bem.server_stats(), bem.server_kernel_stats()


def roofline(kstats, workload="icosphere6"):
    """Roofline of the dominant kernel: the resident (persistent) launches
    when the server served its batches that way, else the launched kernel
    with the most device time."""
    main = list(kstats)
    if not main:
        return None, None
    resident = [k for k in main if k.get("persistent")]
    dom = max(resident or main, key=lambda k: k["seconds"])
    flops = dom["pair_evals"] * FLOPS_PER_EVAL[(dom["op"], dom["space"])]
    per_launch = flops / dom["launches"]
    mean_ev = dom["seconds_events"] / dom["launches"]    # HIP events around the launch, on its stream
    mean_dc = dom["seconds"] / dom["launches"]           # first workgroup start to last workgroup end
    achieved = per_launch / mean_ev / 1e12
    traffic = None
    blocks_per_launch = dom["blocks"] / dom["launches"]
    if os.path.exists(traffic_file(workload)):
        with open(traffic_file(workload)) as f:
            t = json.load(f)
        # per block of entry work: the resident and the launched kernel run the
        # same per-block code (one block per workgroup when launched)
        if t.get("kernel_source_hash") == kernel_source_hash() and "bytes_per_workgroup" in t:
            traffic = t["bytes_per_workgroup"] * blocks_per_launch
    # algorithmic bytes per entry of the measurement plan (P1, 6-point rule):
    # two trial triangles of 36 B of vertex coordinates, a 4-byte index and a
    # 4-byte FP32 output
    alg_bytes = 80.0 * dom["entries"] / dom["launches"]
    name = "%s%s_f%s<op=%d,Q=%d>" % ("kp_" if dom.get("persistent") else "k_",
                                     KERNEL_NAMES[dom["space"]][2:], "32" if dom["prec"] == 1 else "64",
                                     dom["op"], dom["quad_points"])
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_FP32_PACKED / 1e12, 1),
            "unit": "TFLOP/s", "frac": round(achieved * 1e12 / PEAK_FP32_PACKED, 4), "traffic": traffic,
            "kernel": name, "persistent": bool(dom.get("persistent")), "launches": dom["launches"],
            "mean_launch_us": round(mean_ev * 1e6, 2),
            "workgroups_per_launch": round(dom["workgroups"] / dom["launches"], 1),
            "blocks_per_launch": round(blocks_per_launch, 1),
            "mean_launch_us_device_clock": round(mean_dc * 1e6, 2),
            "frac_device_clock": round(per_launch / mean_dc / PEAK_FP32_PACKED, 4),
            "flops_per_launch": per_launch, "flops_per_eval": FLOPS_PER_EVAL[(dom["op"], dom["space"])],
            "executed_flops_per_eval": FLOPS_EXECUTED[(dom["op"], dom["space"])],
            "executed_tflops": round(dom["pair_evals"] * FLOPS_EXECUTED[(dom["op"], dom["space"])] /
                                     dom["launches"] / mean_ev / 1e12, 3),
            "frac_of_unpacked_fp32_peak": round(achieved * 1e12 / PEAK_FP32_VALU, 4),
            "algorithmic_bytes_per_launch": alg_bytes,
            "traffic_over_algorithmic": round(traffic / alg_bytes, 3) if traffic else None}
    return roof, dom


def cpu_baseline(bem, inputs, mesh, xyz, tri, seconds, ops):
    """FP64 oracle on a seeded sample of the benchmark's ACA row/column
    requests (the step's operators in turn, P1), all host threads; stops
    after `seconds`.  Also returns the largest FP32-vs-oracle normwise error
    on that sample."""
    import numpy as np
    import oracle

    om = oracle.OracleMesh(xyz, tri, 6)
    perm, ranges, blocks = bem.partition(xyz, tri, bem.P1, 100, 1.0)
    adm = blocks[blocks[:, 2] == 1]
    rng = inputs.rng(inputs.SEED_SAMPLING)
    entries = 0
    spent = 0.0
    nreq = 0
    worst = 0.0
    while spent < seconds:
        b = adm[int(rng.integers(adm.shape[0]))]
        rows = perm[ranges[b[0], 0]:ranges[b[0], 1]]
        cols = perm[ranges[b[1], 0]:ranges[b[1], 1]]
        op = ops[nreq % len(ops)]   # the same ids in both modules
        if nreq % 4 < 2:
            r, c = rows[int(rng.integers(rows.size)):][:1], cols
        else:
            r, c = rows, cols[int(rng.integers(cols.size)):][:1]
        t0 = time.perf_counter()
        ref = om.entries(op, oracle.P1, 0.0, r, c)
        spent += time.perf_counter() - t0
        entries += ref.size
        nreq += 1
        got = bem.eval_entries(mesh, op, bem.P1, 0.0, r, c, prec=bem.FP32, near=bem.NEAR_ERROR)
        worst = max(worst, float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))
    return {"value": entries / spent, "unit": "entries/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"{nreq} ACA row/column requests ({'/'.join(sorted(set(OP_LABEL[o] for o in ops)))}, P1) of "
                      f"seeded admissible blocks of "
                      f"the same partition, {entries} entries, {spent:.1f} s"}, worst


def cpu_hmatrix(inputs, xyz, tri, ops, fraction, tol=1e-5, max_rank=200):
    """CPU-only H-matrix assembly driven by the FP64 oracle: the oracle's
    partition (leaf 100, eta 1) and its ACA (Algorithm ACA, Section 2.1) with
    the oracle's FP64 rows and columns on all host threads, over a seeded
    fraction of the admissible blocks of each operator; the time for every
    admissible block is extrapolated by the blocks' summed dimensions (ACA
    work goes as rank x (m + n))."""
    import numpy as np
    import oracle
    from oracle import aca as oaca
    from oracle import tree as otree

    om = oracle.OracleMesh(xyz, tri, 6)
    t0 = time.perf_counter()
    nodes, leaves = otree.partition(xyz, tri, oracle.P1, 100, 1.0)
    t_part = time.perf_counter() - t0
    adm = [(t, s) for t, s, a in leaves if a]
    if not adm:
        raise ValueError("the partition has no admissible block")
    rng = inputs.rng(inputs.SEED_SAMPLING)
    pick = rng.choice(len(adm), size=max(1, int(round(fraction * len(adm)))), replace=False)
    mn_all = float(sum(nodes[t].idx.size + nodes[s].idx.size for t, s in adm))
    out = {"kind": "oracle", "cores": oracle.max_threads(), "partition_seconds": t_part,
           "admissible_blocks": len(adm), "sampled_blocks": int(pick.size), "ops": {}}
    total = 0.0
    for op in ops:
        entries, spent, rank_sum, mn = 0, 0.0, 0, 0
        for i in pick:
            t, s = adm[int(i)]
            rows = nodes[t].idx.astype(np.int32)
            cols = nodes[s].idx.astype(np.int32)
            count = [0]

            def get_row(k, rows=rows, cols=cols, count=count):
                count[0] += cols.size
                return om.entries(op, oracle.P1, 0.0, rows[k:k + 1], cols)[0]

            def get_col(k, rows=rows, cols=cols, count=count):
                count[0] += rows.size
                return om.entries(op, oracle.P1, 0.0, rows, cols[k:k + 1])[:, 0]

            ts = time.perf_counter()
            U, V, _, _ = oaca.aca(get_row, get_col, rows.size, cols.size, tol, max_rank)
            spent += time.perf_counter() - ts
            entries += count[0]
            rank_sum += U.shape[1]
            mn += rows.size + cols.size
        full = spent * mn_all / mn
        total += full
        out["ops"][OP_LABEL[op]] = {"sampled_seconds": spent, "sampled_entries": entries,
                                    "entries_per_s": entries / spent, "mean_rank": rank_sum / pick.size,
                                    "extrapolated_seconds_all_admissible_blocks": full}
    out["extrapolated_seconds"] = total
    out["sample"] = (f"{pick.size} of {len(adm)} admissible blocks per operator (seed {inputs.SEED_SAMPLING}), "
                     f"oracle ACA tol {tol}, FP64 oracle rows and columns on {out['cores']} threads; time for all "
                     "admissible blocks extrapolated by summed block dimensions")
    return out


def dense_run(bem, mesh, idx, ops, prec, chunk):
    n = idx.size
    tickets = [bem.submit(mesh, op, bem.P1, 0.0, idx[i:i + chunk], idx, prec=prec)
               for op in ops for i in range(0, n, chunk)]
    for t in tickets:
        t.wait()
    return tickets


# Algorithmic flops per kernel evaluation of a pair's 3 x 3 local matrix:
# the kernel core of the measurement plan's P0 count (without its weighted
# accumulation), three test-basis accumulations per point pair, and the nine
# trial-basis products per trial point spread over its Q test points
# (Q = 6: 18 / Q = 3 flops, complex twice that).
FLOPS_PER_EVAL_DENSE = {0: 9 + 6 + 3, 1: 17 + 6 + 3, 2: 16 + 12 + 6, 3: 29 + 12 + 6}


def dense_main(args):
    """Dense weak-form assembly (the paper's first benchmark): every entry of
    the P1 matrix, all regular pairs (vertex-sharing pairs skipped), by
    triangle pairs (bem_eval_dense: each pair's local matrix once, 144 kernel
    evaluations per entry), beside the same matrix through the request server's
    star kernels (each pair once per test vertex, 432 per entry)."""
    import numpy as np
    import torch
    os.environ.setdefault("BEM_SERVER_STREAMS", "1")
    from paper_1711_01897_amd import bem, inputs
    xyz, tri = inputs.icosphere(args.dense)
    n = xyz.shape[0]
    mesh = bem.mesh_create(xyz, tri, 6)
    ops = step_ops(args)
    # rows and columns in the cluster-tree order (the matrix is the same,
    # permuted): a panel's row stars then share their triangles
    idx = bem.partition(xyz, tri, bem.P1, 100, 1.0)[0].astype(np.int32)

    def run(prec):
        stats = []
        outs = []
        for op in ops:
            out, st = bem.eval_dense(mesh, op, bem.P1, 0.0, idx, idx, prec=prec, near=bem.NEAR_SKIP, stats=True)
            stats.append(st)
            outs.append(out)
        return outs, stats

    for _ in range(args.warmup):
        run(bem.FP32)
    torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        last, stats = run(bem.FP32)
        times.append(time.perf_counter() - t0)
    dt = sum(times)
    entries = len(ops) * n * n * args.steps
    # roofline of the local-matrix kernel: its first panel, HIP events
    st0, op0 = stats[0], ops[0]
    flops = st0["first_pairs"] * 36 * FLOPS_PER_EVAL_DENSE[op0 if op0 < 4 else 1]
    achieved = flops / st0["first_local_seconds"] if st0["first_local_seconds"] > 0 else 0.0
    roof = {"bound": "alu", "achieved": round(achieved / 1e12, 3), "peak": round(PEAK_FP32_PACKED / 1e12, 1),
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_PACKED, 4), "traffic": None,
            "kernel": f"k_local_f32<op={op0},Q=6>", "pairs_per_launch": st0["first_pairs"],
            "launch_us": round(st0["first_local_seconds"] * 1e6, 1),
            "gather_us": round(st0["first_gather_seconds"] * 1e6, 1),
            "flops_per_eval": FLOPS_PER_EVAL_DENSE[op0 if op0 < 4 else 1],
            "frac_of_unpacked_fp32_peak": round(achieved / PEAK_FP32_VALU, 4)}
    evals_per_entry = sum(st["pairs"] for st in stats) * 36 / (len(ops) * n * n)
    fp64 = None
    if not args.no_fp64:
        t1 = time.perf_counter()
        run(bem.FP64)
        dt64 = time.perf_counter() - t1
        fp64 = {"value": len(ops) * n * n / dt64, "unit": "entries/s", "seconds_per_step": dt64}
    # the same matrix through the request server's star kernels, one step
    star = None
    if not args.no_star:
        chunk = 512
        t2 = time.perf_counter()
        dense_run(bem, mesh, idx, ops, bem.FP32, chunk)
        dts = time.perf_counter() - t2
        star = {"value": len(ops) * n * n / dts, "unit": "entries/s", "evals_per_entry": 432,
                "requests": f"{chunk}-row requests through the request server"}
    worst = None
    if not args.no_cpu_baseline:
        import oracle
        om = oracle.OracleMesh(xyz, tri, 6)
        pos = np.arange(0, n, max(1, n // 4))[:4]   # row positions in idx
        worst = 0.0
        for k, op in enumerate(ops):
            ref = om.entries(op, oracle.P1, 0.0, idx[pos], idx)
            worst = max(worst, float(np.max(np.abs(last[k][pos] - ref)) / np.max(np.abs(ref))))
    line = {
        "metric": "dense weak-form entries/sec FP32 vs FP64",
        "value": entries / dt, "unit": "entries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"dense P1 matrix of the Laplace {' + '.join(OP_LABEL[o] for o in ops)} operator(s), "
                               f"icosphere level {args.dense} ({tri.shape[0]} triangles, {n} vertices), 6-point rule, "
                               "vertex-sharing pairs skipped, rows and columns in cluster-tree order, each triangle "
                               "pair's local matrix once (bem_eval_dense), FP32 compensated entries, results in host "
                               "memory", "panels": stats[0]["panels"],
                   "kernel_evals_per_entry": round(evals_per_entry, 1)},
        "step_seconds_median": sorted(times)[len(times) // 2], "step_seconds_min": min(times),
        "fp64": fp64, "fp32_over_fp64": (entries / dt / fp64["value"]) if fp64 else None,
        "star_kernel_path": star, "pair_over_star": (entries / dt / star["value"]) if star else None,
        "max_rel_err_sampled": worst, "roofline": roof,
    }
    print(json.dumps(line))


def complete_main(args):
    """Complete P0 H-matrix (leaf 100, eta 1, ACA tol 1e-8, FP64):
    admissible leaves by ACA, dense leaves with their vertex-sharing pairs
    integrated on the device; timed against the same assembly with the
    singular pairs skipped."""
    import numpy as np
    from paper_1711_01897_amd import bem, inputs
    xyz, tri = inputs.icosphere(args.complete)
    mesh = bem.mesh_create(xyz, tri, 6)
    nt = tri.shape[0]
    op = {"laplace_slp": bem.LAPLACE_SLP, "laplace_dlp": bem.LAPLACE_DLP, "helmholtz_slp": bem.HELMHOLTZ_SLP,
          "helmholtz_dlp": bem.HELMHOLTZ_DLP, "laplace_hyps": bem.LAPLACE_HYPS,
          "helmholtz_hyps": bem.HELMHOLTZ_HYPS}[args.complete_op]
    k = inputs.wavenumber(xyz, tri, 10.0) if bem.is_complex(op) else 0.0
    space = bem.P1 if args.complete_space == "p1" else bem.P0

    def assemble(mode):
        t0 = time.perf_counter()
        H = bem.hmat_assemble(mesh, op, space, k, leaf_size=100, eta=1.0, aca_tol=1e-8,
                              max_rank=200, n_workers=args.workers, blocks_per_worker=args.blocks_per_worker,
                              prec=bem.FP64, dense_mode=mode)
        dt = time.perf_counter() - t0
        st = H.stats()
        H.destroy()
        return dt, st

    for _ in range(args.warmup):
        assemble(2)
    t2 = min(assemble(2)[0] for _ in range(args.steps))
    t1, st = min((assemble(1) for _ in range(args.steps)), key=lambda r: r[0])
    # vertex-sharing pairs by the number of shared vertices (3 identical, 2 common edge, 1 common vertex)
    stars = [[] for _ in range(xyz.shape[0])]
    for t, (a, b, c) in enumerate(tri.tolist()):
        stars[a].append(t), stars[b].append(t), stars[c].append(t)
    kinds = {1: 0, 2: 0, 3: 0}
    for t, verts in enumerate(tri.tolist()):
        vs = set(verts)
        for s in set(stars[verts[0]] + stars[verts[1]] + stars[verts[2]]):
            kinds[len(vs.intersection(tri[s].tolist()))] += 1
    if op in (bem.LAPLACE_DLP, bem.HELMHOLTZ_DLP):
        kinds[3] = 0   # the double layer of a flat triangle on itself vanishes: no items
    # algorithmic flops of the Laplace single-layer singular-pair kernel: 14 per kernel evaluation (difference
    # vector 6, |c|^2 5, rsqrt 1, weighted sum 2); evaluations per pair 96 (identical), 1024 (common edge),
    # 8192 (common vertex)
    near_flops = 14 * (96 * kinds[3] + 1024 * kinds[2] + 8192 * kinds[1]) \
        if (op == bem.LAPLACE_SLP and space == bem.P0) else None
    label = {bem.LAPLACE_SLP: "Laplace single layer", bem.LAPLACE_DLP: "Laplace double layer",
             bem.HELMHOLTZ_SLP: "Helmholtz single layer", bem.HELMHOLTZ_DLP: "Helmholtz double layer",
             bem.LAPLACE_HYPS: "Laplace hypersingular operator",
             bem.HELMHOLTZ_HYPS: "Helmholtz hypersingular operator"}[op]
    line = {
        "metric": f"complete H-matrix assembly seconds ({args.complete_space.upper()} {label}, FP64)",
        "value": t2, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "higher_is_better": False, "scaling": "strong", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"icosphere level {args.complete} ({nt} triangles), leaf 100, eta 1.0, ACA tol 1e-8, "
                               "dense leaves complete (singular pairs on the device)"
                               + (f", k = {k:.4g} (10 elements per wavelength)" if k else ""),
                   "admissible_blocks": st["admissible_blocks"], "dense_blocks": st["dense_blocks"],
                   "dense_entries": st["dense_entries"], "aca_entries": st["aca_entries"]},
        "seconds_without_singular_pairs": t1, "singular_pairs": sum(kinds.values()),
        "singular_pairs_by_shared_vertices": {str(s): v for s, v in kinds.items()},
        "singular_kernel_flops_per_assembly": near_flops,
        "singular_pairs_per_second_marginal": sum(kinds.values()) / max(t2 - t1, 1e-9),
    }
    print(json.dumps(line))


def gpu_telemetry():
    """GPU temperature and clocks (the paper saw thermal down-clocking in its
    runs, Section 5), or None where the management library is unavailable."""
    try:
        import amdsmi
        amdsmi.amdsmi_init()
        try:
            handles = amdsmi.amdsmi_get_processor_handles()
            if not handles:
                return None
            h = handles[0]
            out = {}
            try:
                out["edge_temp_c"] = amdsmi.amdsmi_get_temp_metric(h, amdsmi.AmdSmiTemperatureType.EDGE,
                                                                   amdsmi.AmdSmiTemperatureMetric.CURRENT)
            except Exception:
                pass
            try:
                out["hotspot_temp_c"] = amdsmi.amdsmi_get_temp_metric(h, amdsmi.AmdSmiTemperatureType.HOTSPOT,
                                                                      amdsmi.AmdSmiTemperatureMetric.CURRENT)
            except Exception:
                pass
            try:
                c = amdsmi.amdsmi_get_clock_info(h, amdsmi.AmdSmiClkType.GFX)
                out["gfx_clock_mhz"] = c.get("clk")
                out["gfx_clock_max_mhz"] = c.get("max_clk")
            except Exception:
                pass
            try:
                act = amdsmi.amdsmi_get_gpu_activity(h)
                out["gfx_activity_pct"] = act.get("gfx_activity")
            except Exception:
                pass
            return out or None
        finally:
            amdsmi.amdsmi_shut_down()
    except Exception:
        return None


def host_cores():
    """Cores this process may use (affinity), the machine's logical CPUs and
    the CPU model (from /proc/cpuinfo, as lscpu reports it)."""
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    model = cores_per_socket = siblings = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                key = line.split(":", 1)[0].strip()
                val = line.split(":", 1)[1].strip() if ":" in line else ""
                if key == "model name" and model is None:
                    model = val
                elif key == "cpu cores" and cores_per_socket is None:
                    cores_per_socket = int(val)
                elif key == "siblings" and siblings is None:
                    siblings = int(val)
    except (OSError, ValueError):
        pass
    smt = (siblings // cores_per_socket) if (siblings and cores_per_socket) else None
    return {"usable": usable, "logical": os.cpu_count(), "model": model, "threads_per_core": smt}


CYL = {"leaf": 16, "eta": 1.0, "tol": 1e-5, "max_block": 4096, "max_rank": 200}


def cylinder_workload_name(nt, nv, args):
    return (f"served Laplace single layer, P1, capped cylinder R=1 L=16 ({nt} triangles, {nv} vertices, +-1% "
            f"jitter seed 0), 6-point rule, H-matrix leaf {CYL['leaf']}, eta {CYL['eta']}, largest block "
            f"{CYL['max_block']}, ACA tol {CYL['tol']}, {args.workers} host ACA workers x {args.blocks_per_worker} "
            "blocks, Poisson block arrivals (seed 1), every ACA row/column on the GPU through the request server, "
            "FP32 compensated entries")


def poisson_arrivals(rng, n, rate):
    """n arrival times (s) of a Poisson process of the given rate, first at t=0."""
    import numpy as np
    gaps = rng.exponential(1.0 / rate, size=n)
    gaps[0] = 0.0
    return np.cumsum(gaps)


def serve_leg(bem, inputs, plan, segs, prec, args, label):
    """Warm-up segments closed-loop (capacity), then the timed segments as
    Poisson streams at args.load x capacity, then the load sweep."""
    import numpy as np
    import torch
    nw = args.warmup
    warm = []
    for i in range(nw):
        t0 = time.perf_counter()
        st = plan.run(segs[i], None, prec)
        warm.append((st, time.perf_counter() - t0))
    use = warm[1:] if len(warm) > 1 else warm
    if use:
        cap_blocks = sum(w[0]["blocks"] for w in use) / sum(w[1] for w in use)
        cap_entries = sum(w[0]["entries"] for w in use) / sum(w[1] for w in use)
    else:
        t0 = time.perf_counter()
        st = plan.run(segs[0][: max(1, len(segs[0]) // 4)], None, prec)
        dt = time.perf_counter() - t0
        cap_blocks, cap_entries = st["blocks"] / dt, st["entries"] / dt
    rate = args.load * cap_blocks
    rng = inputs.rng(inputs.SEED_ARRIVALS)
    bem.server_stats(reset=True)
    bem.server_kernel_stats(reset=True)
    tel0 = gpu_telemetry()
    torch.cuda.synchronize()
    steps = []
    ru0 = resource.getrusage(resource.RUSAGE_SELF)
    t_all = time.perf_counter()
    for i in range(args.steps):
        seg = segs[nw + i]
        arr = poisson_arrivals(rng, len(seg), rate)
        t0 = time.perf_counter()
        st = plan.run(seg, arr, prec)
        dt = time.perf_counter() - t0
        steps.append((st, dt))
        print(f"[bench] {label} step {i}: {st['blocks']} blocks {st['entries']} entries {dt:.3f} s", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_all
    ru1 = resource.getrusage(resource.RUSAGE_SELF)
    tel1 = gpu_telemetry()
    sst = bem.server_stats()
    kst = bem.server_kernel_stats()
    ent = sum(x[0]["entries"] for x in steps)
    secs = sum(x[1] for x in steps)
    per = sorted(x[0]["entries"] / x[1] for x in steps)
    out = {
        "value": ent / wall, "entries_per_step": ent // max(1, len(steps)),
        "requests_per_step": sum(x[0]["requests"] for x in steps) // max(1, len(steps)),
        "blocks_per_step": sum(x[0]["blocks"] for x in steps) // max(1, len(steps)),
        "seconds_per_step": secs / max(1, len(steps)), "wall": wall,
        "step_entries_per_s_median": per[len(per) // 2] if per else None,
        "step_entries_per_s_min": per[0] if per else None,
        "rank_sum": sum(x[0]["rank_sum"] for x in steps), "rank_max": max((x[0]["rank_max"] for x in steps),
                                                                           default=0),
        "mean_rank": sum(x[0]["rank_sum"] for x in steps) / max(1, sum(x[0]["blocks"] for x in steps)),
        "capacity_blocks_per_s": cap_blocks, "capacity_entries_per_s": cap_entries, "arrival_rate_blocks_per_s": rate,
        "mean_block_start_delay_ms": 1e3 * sum(x[0]["mean_start_delay"] * x[0]["blocks"] for x in steps) /
        max(1, sum(x[0]["blocks"] for x in steps)),
        "mean_block_ms": 1e3 * sum(x[0]["mean_block_seconds"] * x[0]["blocks"] for x in steps) /
        max(1, sum(x[0]["blocks"] for x in steps)),
        "latency_p50_ms": sst["latency_p50"] * 1e3, "latency_p99_ms": sst["latency_p99"] * 1e3,
        "sst": sst, "kst": kst, "telemetry": {"before": tel0, "after": tel1},
        # host CPU time of the whole process over the timed steps (all threads)
        "host_cpu": {"user_seconds": ru1.ru_utime - ru0.ru_utime, "system_seconds": ru1.ru_stime - ru0.ru_stime,
                     "cores_busy": (ru1.ru_utime - ru0.ru_utime + ru1.ru_stime - ru0.ru_stime) / wall,
                     "voluntary_switches": ru1.ru_nvcsw - ru0.ru_nvcsw,
                     "involuntary_switches": ru1.ru_nivcsw - ru0.ru_nivcsw},
    }
    sweep = []
    loads = [float(x) for x in args.sweep.split(",") if x.strip()] if args.sweep else []
    for j, ld in enumerate(loads):
        seg = segs[(nw + args.steps + j) % len(segs)]
        arr = poisson_arrivals(rng, len(seg), ld * cap_blocks)
        bem.server_stats(reset=True)
        t0 = time.perf_counter()
        st = plan.run(seg, arr, prec)
        dt = time.perf_counter() - t0
        ss = bem.server_stats()
        sweep.append({"load": ld, "entries_per_s": st["entries"] / dt, "latency_p50_ms": ss["latency_p50"] * 1e3,
                      "latency_p99_ms": ss["latency_p99"] * 1e3,
                      "mean_block_start_delay_ms": st["mean_start_delay"] * 1e3})
    out["latency_vs_load"] = sweep
    return out


def cylinder_cpu_baseline(bem, inputs, plan, mesh, xyz, tri, seconds):
    """FP64 oracle on a seeded sample of ACA row/column requests of the
    plan's admissible blocks (seed 3): all usable host threads for most of
    the budget, one thread for the rest.  Also returns the largest FP32
    normwise error of the device on the same requests."""
    import numpy as np
    import oracle

    om = oracle.OracleMesh(xyz, tri, 6)
    nb = plan.info()["blocks"]
    rng = inputs.rng(inputs.SEED_SAMPLING)
    worst = 0.0

    def sample(budget, nthreads):
        nonlocal worst
        spent, entries, nreq = 0.0, 0, 0
        while spent < budget:
            rows, cols = plan.block(int(rng.integers(nb)))
            if nreq % 2 == 0:
                r, c = rows[int(rng.integers(rows.size)):][:1], cols
            else:
                r, c = rows, cols[int(rng.integers(cols.size)):][:1]
            t0 = time.perf_counter()
            ref = om.entries(oracle.LAPLACE_SLP, oracle.P1, 0.0, r, c, nthreads=nthreads)
            spent += time.perf_counter() - t0
            entries += ref.size
            nreq += 1
            got = bem.eval_entries(mesh, bem.LAPLACE_SLP, bem.P1, 0.0, r, c, prec=bem.FP32, near=bem.NEAR_ERROR)
            worst = max(worst, float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))
        return entries / spent, nreq, entries, spent

    cores = host_cores()
    all_rate, n_all, e_all, s_all = sample(0.75 * seconds, 0)
    one_rate, n_one, e_one, s_one = sample(0.25 * seconds, 1)
    return {"value": all_rate, "unit": "entries/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"{n_all} ACA row/column requests of seeded admissible blocks of the served cylinder "
                      f"partition (Laplace single layer, P1), {e_all} entries, {s_all:.1f} s on "
                      f"{oracle.max_threads()} threads; {n_one} requests, {e_one} entries, {s_one:.1f} s on 1",
            "one_core_value": one_rate, "host": cores}, worst


def kernel_entries_rate(kstats):
    """Entries per second of entry-kernel time (HIP-event launch brackets) of
    the variant with the most device time: the GPU path's own rate, apart
    from the host loop around it."""
    main = [k for k in kstats if not k.get("persistent")]
    if not main:
        return None
    dom = max(main, key=lambda k: k["seconds"])
    return dom["entries"] / dom["seconds_events"] if dom["seconds_events"] > 0 else None


def cylinder_main(args):
    import numpy as np
    from paper_1711_01897_amd import bem, inputs

    t0 = time.perf_counter()
    xyz, tri = inputs.capped_cylinder()
    mesh = bem.mesh_create(xyz, tri, 6)
    print(f"[bench] mesh {tri.shape[0]} triangles / {xyz.shape[0]} vertices resident "
          f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    plan = bem.aca_plan_create(mesh, bem.LAPLACE_SLP, bem.P1, 0.0, leaf_size=CYL["leaf"], eta=CYL["eta"],
                               aca_tol=CYL["tol"], max_rank=CYL["max_rank"], n_workers=args.workers,
                               blocks_per_worker=args.blocks_per_worker, prec=bem.FP32, max_block=CYL["max_block"])
    info = plan.info()
    print(f"[bench] plan: {info['blocks']} admissible blocks, set-up {info['setup_seconds']:.1f} s", file=sys.stderr,
          flush=True)
    order = inputs.rng(inputs.SEED_REQUESTS).permutation(info["blocks"]).astype(np.int64)
    segs = np.array_split(order, args.warmup + args.steps)
    f32 = serve_leg(bem, inputs, plan, segs, bem.FP32, args, "fp32")
    roof, dom = roofline(f32["kst"], "cylinder")
    fp64 = None
    if not args.no_fp64:
        f64 = serve_leg(bem, inputs, plan, segs, bem.FP64, args, "fp64")
        fp64 = {k: f64[k] for k in ("value", "entries_per_step", "requests_per_step", "seconds_per_step",
                                    "step_entries_per_s_median", "step_entries_per_s_min", "mean_rank", "rank_max",
                                    "latency_p50_ms", "latency_p99_ms", "capacity_entries_per_s",
                                    "arrival_rate_blocks_per_s", "latency_vs_load")}
        fp64["unit"] = "entries/s"
        fp64["kernel_entries_per_s"] = kernel_entries_rate(f64["kst"])
    kernel_rate = {"fp32": kernel_entries_rate(f32["kst"]), "fp64": fp64["kernel_entries_per_s"] if fp64 else None}
    if kernel_rate["fp32"] and kernel_rate["fp64"]:
        kernel_rate["fp32_over_fp64"] = kernel_rate["fp32"] / kernel_rate["fp64"]
    cpu, worst = (None, None)
    if not args.no_cpu_baseline:
        cpu, worst = cylinder_cpu_baseline(bem, inputs, plan, mesh, xyz, tri, args.cpu_seconds)
        cpu["speedup_S"] = f32["value"] / cpu["value"]
        cpu["speedup_S_one_core"] = f32["value"] / cpu["one_core_value"]
        print(f"[bench] cpu baseline {cpu['value']:.3e} entries/s on {cpu['cores']} threads", file=sys.stderr,
              flush=True)
    sst = f32["sst"]
    line = {
        "metric": "weak-form entries/sec FP32 vs FP64 at stated rel err; p50/p99 ACA request latency",
        "value": f32["value"], "unit": "entries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": f32["wall"] / max(1, args.steps) * 1e3, "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": cylinder_workload_name(tri.shape[0], xyz.shape[0], args),
                   "admissible_blocks": info["blocks"], "blocks_per_step": f32["blocks_per_step"],
                   "aca_entries_per_step": f32["entries_per_step"], "aca_requests_per_step": f32["requests_per_step"],
                   "mean_rank": f32["mean_rank"], "max_rank": f32["rank_max"], "workers": args.workers,
                   "blocks_per_worker": args.blocks_per_worker, "offered_load": args.load,
                   "arrival_rate_blocks_per_s": f32["arrival_rate_blocks_per_s"],
                   "plan_setup_seconds": info["setup_seconds"]},
        "latency_p50_ms": f32["latency_p50_ms"], "latency_p99_ms": f32["latency_p99_ms"],
        "step_entries_per_s_median": f32["step_entries_per_s_median"],
        "step_entries_per_s_min": f32["step_entries_per_s_min"],
        "capacity_entries_per_s": f32["capacity_entries_per_s"],
        "mean_block_start_delay_ms": f32["mean_block_start_delay_ms"], "mean_block_ms": f32["mean_block_ms"],
        "latency_vs_load": f32["latency_vs_load"],
        "fused_launch_batches": sst["batches"], "requests_per_batch": sst["requests"] / max(1, sst["batches"]),
        "server_seconds_per_step": {"dispatch": sst["dispatch_seconds"] / args.steps,
                                    "dispatch_hip_calls": sst["dispatch_hip_seconds"] / args.steps,
                                    "complete": sst["complete_seconds"] / args.steps,
                                    "event_wait": sst["wait_seconds"] / args.steps,
                                    "entry_kernels": sst["kernel_seconds"] / args.steps},
        "request_latency_legs_us": {k: round(sst["mean_%s_seconds" % k] * 1e6, 1)
                                    for k in ("queue", "stage", "device", "complete")},
        "kernel_busy_fraction": sst["kernel_seconds"] / f32["wall"] if f32["wall"] > 0 else None,
        "fp64": fp64, "fp32_over_fp64": (f32["value"] / fp64["value"]) if fp64 else None,
        "kernel_entries_per_s": kernel_rate,
        "max_rel_err_sampled": worst, "gpu_telemetry": f32["telemetry"],
        "host_cpu": dict(f32["host_cpu"], **host_cores()),
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    plan.destroy()
    mesh.destroy()


def timed_runs(fn, warmup, steps):
    """warmup untimed calls, then `steps` timed ones: (times, last result)."""
    for _ in range(warmup):
        fn()
    times, res = [], None
    for _ in range(steps):
        t0 = time.perf_counter()
        res = fn()
        times.append(time.perf_counter() - t0)
    return times, res


def spheroid_main(args):
    """H-matrix of the Helmholtz single layer, P0, 4-point rule, on the
    262,186-triangle 10:1:1 prolate spheroid at 10 elements per wavelength
    (leaf 100, eta 1, ACA tol 1e-4), one assembly per step: complex64
    entries against complex128 entries, both by the measurement protocol
    (warm-ups, then timed runs; median and min)."""
    import numpy as np
    from paper_1711_01897_amd import bem, inputs
    xyz, tri = inputs.spheroid(10.0, 1.0, 262144)
    mesh = bem.mesh_create(xyz, tri, 4)
    k = inputs.wavenumber(xyz, tri, 10.0)
    res = {}
    for prec in (bem.FP32, bem.FP64):
        def one():
            H = bem.hmat_assemble(mesh, bem.HELMHOLTZ_SLP, bem.P0, k, leaf_size=100, eta=1.0, aca_tol=1e-4,
                                  max_rank=300, n_workers=args.workers, blocks_per_worker=args.blocks_per_worker,
                                  prec=prec, dense_mode=0)
            st = H.stats()
            H.destroy()
            return st
        bem.server_stats(reset=True)
        bem.server_kernel_stats(reset=True)
        times, st = timed_runs(one, args.warmup, args.steps)
        sst = bem.server_stats()
        res[prec] = {"entries_per_s": st["aca_entries"] / float(np.median(times)),
                     "seconds_median": float(np.median(times)), "seconds_min": min(times),
                     "aca_entries": st["aca_entries"], "aca_requests": st["aca_requests"],
                     "mean_rank": st["rank_sum"] / max(1, st["admissible_blocks"]), "rank_max": st["rank_max"],
                     "latency_p50_ms": sst["latency_p50"] * 1e3, "latency_p99_ms": sst["latency_p99"] * 1e3,
                     "kst": bem.server_kernel_stats()}
        print(f"[bench] spheroid prec {prec}: median {res[prec]['seconds_median']:.3f} s", file=sys.stderr, flush=True)
    for prec in (bem.FP32, bem.FP64):
        res[prec]["kernel_entries_per_s"] = kernel_entries_rate(res[prec]["kst"])
    roof, _ = roofline(res[bem.FP32].pop("kst"), "spheroid")
    res[bem.FP64].pop("kst")
    f32, f64 = res[bem.FP32], res[bem.FP64]
    line = {"metric": "weak-form entries/sec complex64 vs complex128 (H-matrix ACA assembly)",
            "value": f32["entries_per_s"], "unit": "entries/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": f32["seconds_median"] * 1e3, "higher_is_better": True,
            "scaling": "strong", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
            "config": {"workload": f"Helmholtz single layer, P0, 4-point rule, 10:1:1 spheroid ({tri.shape[0]} "
                                   f"triangles), k = {k:.4g} (10 elements per wavelength), H-matrix leaf 100, eta 1, "
                                   f"ACA tol 1e-4, {args.workers} workers"},
            "fp32": f32, "fp64": f64, "fp32_over_fp64": f32["entries_per_s"] / f64["entries_per_s"],
            "seconds_fp32_over_fp64": f32["seconds_median"] / f64["seconds_median"], "roofline": roof,
            "gpu_telemetry": gpu_telemetry()}
    print(json.dumps(line))


def mix_main(args):
    """Served mixed Helmholtz workload: 8 meshes (icospheres with 5,120 to
    327,680 triangles, 10:1:1 spheroids with ~10k to ~400k) x 4 wavenumbers
    (2, 5, 10, 20 elements per wavelength), Helmholtz single layer, P0,
    4-point rule, complex64, ACA plans with leaf 16, eta 1, tol 1e-4.  All 32
    (mesh, k) instances are served together (bem_aca_plans_run): one pool of
    32 host ACA workers takes blocks from every instance through the one
    device queue.  A seeded share (--mix-fraction, seed 2) of the admissible
    blocks of all instances, in that seeded order, is cut into warm-up +
    timed segments; the warm-up segments run closed-loop and give the capacity, each
    timed segment is a Poisson stream of block arrivals (seed 1) at
    args.load x capacity.  The same with complex128 entries is the FP64 leg."""
    import numpy as np
    from paper_1711_01897_amd import bem, inputs
    meshes = [("icosphere", 4), ("icosphere", 5), ("icosphere", 6), ("icosphere", 7),
              ("spheroid", 10000), ("spheroid", 40000), ("spheroid", 160000), ("spheroid", 400000)]
    geo = [inputs.icosphere(size) if kind == "icosphere" else inputs.spheroid(10.0, 1.0, size)
           for kind, size in meshes]
    inst = []
    for (kind, size), (xyz, tri) in zip(meshes, geo):
        mesh = bem.mesh_create(xyz, tri, 4)
        for epw in (2.0, 5.0, 10.0, 20.0):
            k = inputs.wavenumber(xyz, tri, epw)
            plan = bem.aca_plan_create(mesh, bem.HELMHOLTZ_SLP, bem.P0, k, leaf_size=16, eta=1.0, aca_tol=1e-4,
                                       max_rank=200, n_workers=1, blocks_per_worker=1, prec=bem.FP32)
            inst.append({"mesh": mesh, "plan": plan, "k": k, "name": f"{kind}{size}@{epw:g}",
                         "blocks": plan.info()["blocks"]})
    plans = [it["plan"] for it in inst]
    pidx = np.concatenate([np.full(it["blocks"], p, dtype=np.int64) for p, it in enumerate(inst)])
    bidx = np.concatenate([np.arange(it["blocks"], dtype=np.int64) for it in inst])
    order = inputs.rng(inputs.SEED_REQUESTS).permutation(pidx.size)
    order = order[:max(1, int(round(args.mix_fraction * order.size)))]
    segs = np.array_split(order, args.warmup + args.steps)
    print(f"[bench] mix: {len(inst)} instances, {pidx.size} admissible blocks, serving {order.size}", file=sys.stderr,
          flush=True)

    def run(seg, arr, prec):
        return bem.aca_plans_run(plans, pidx[seg], bidx[seg], arr, prec, n_workers=args.workers,
                                 blocks_per_worker=args.blocks_per_worker)

    res = {}
    for prec in (bem.FP32, bem.FP64):
        warm = []
        for i in range(args.warmup):
            t0 = time.perf_counter()
            st = run(segs[i], None, prec)
            warm.append((st["blocks"], time.perf_counter() - t0))
        use = warm[1:] if len(warm) > 1 else warm
        cap = sum(w[0] for w in use) / sum(w[1] for w in use) if use else None
        rng = inputs.rng(inputs.SEED_ARRIVALS)
        bem.server_stats(reset=True)
        times, ents, reqs = [], 0, 0
        for i in range(args.steps):
            seg = segs[args.warmup + i]
            arr = poisson_arrivals(rng, seg.size, args.load * cap) if cap else None
            t0 = time.perf_counter()
            st = run(seg, arr, prec)
            times.append(time.perf_counter() - t0)
            ents += st["entries"]
            reqs += st["requests"]
            print(f"[bench] mix prec {prec} step {i}: {st['blocks']} blocks {st['entries']} entries "
                  f"{times[-1]:.3f} s", file=sys.stderr, flush=True)
        sst = bem.server_stats()
        res[prec] = {"entries_per_s": ents / sum(times), "latency_p50_ms": sst["latency_p50"] * 1e3,
                     "latency_p99_ms": sst["latency_p99"] * 1e3,
                     "requests_per_batch": sst["requests"] / max(1, sst["batches"]),
                     "step_seconds_median": float(np.median(times)), "requests_per_step": reqs // args.steps,
                     "entries_per_step": ents // args.steps, "capacity_blocks_per_s": cap}
    # error per (mesh, k) instance against the oracle on seeded ACA rows
    worst = {}
    if not args.no_cpu_baseline:
        import oracle
        rng = inputs.rng(inputs.SEED_SAMPLING)
        cache = {}
        for it in inst:
            key = id(it["mesh"])
            if key not in cache:
                xyz, tri = geo[len(cache)]
                cache[key] = oracle.OracleMesh(xyz, tri, 4)
            om = cache[key]
            e = 0.0
            for _ in range(2):
                rows, cols = it["plan"].block(int(rng.integers(it["blocks"])))
                r = rows[:1]
                got = bem.eval_entries(it["mesh"], bem.HELMHOLTZ_SLP, bem.P0, it["k"], r, cols, prec=bem.FP32,
                                       near=bem.NEAR_ERROR)
                ref = om.entries(oracle.HELMHOLTZ_SLP, oracle.P0, it["k"], r, cols)
                e = max(e, float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))
            worst[it["name"]] = e
    f32, f64 = res[bem.FP32], res[bem.FP64]
    line = {"metric": "weak-form entries/sec FP32 vs FP64 at stated rel err; p50/p99 ACA request latency",
            "value": f32["entries_per_s"], "unit": "entries/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": f32["step_seconds_median"] * 1e3, "higher_is_better": True,
            "scaling": "strong", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
            "config": {"workload": "served Helmholtz single layer, P0, 4-point rule, 8 meshes (icospheres 5,120-"
                                   "327,680 triangles, 10:1:1 spheroids ~10k-400k) x 4 wavenumbers (2, 5, 10, 20 "
                                   "elements per wavelength), ACA plans leaf 16, eta 1, tol 1e-4, one device queue, "
                                   f"one pool of {args.workers} host ACA workers x {args.blocks_per_worker} blocks "
                                   "over all 32 instances, Poisson block arrivals (seed 1) at "
                                   f"{args.load} x the warm-up capacity",
                       "admissible_blocks": int(pidx.size), "blocks_served": int(order.size),
                       "requests_per_step": f32["requests_per_step"],
                       "entries_per_step": f32["entries_per_step"]},
            "latency_p50_ms": f32["latency_p50_ms"], "latency_p99_ms": f32["latency_p99_ms"],
            "requests_per_batch": f32["requests_per_batch"],
            "fp64": f64, "fp32_over_fp64": f32["entries_per_s"] / f64["entries_per_s"],
            "max_rel_err_sampled_per_instance": worst}
    print(json.dumps(line))
    for it in inst:
        it["plan"].destroy()


def sphere3_main(args):
    """The dense P0 Laplace single layer of the level-3 icosphere (1,280
    triangles), FP64 plain path: 1,638,400 entries of which 1,621,820 regular
    (vertex-sharing pairs skipped), one request per step; checked entry by
    entry against the oracle."""
    import numpy as np
    from paper_1711_01897_amd import bem, inputs
    xyz, tri = inputs.icosphere(3)
    mesh = bem.mesh_create(xyz, tri, 6)
    idx = np.arange(tri.shape[0], dtype=np.int32)
    res = {}
    for prec in (bem.FP64, bem.FP32):
        times, A = timed_runs(lambda: bem.eval_entries(mesh, bem.LAPLACE_SLP, bem.P0, 0.0, idx, idx, prec=prec,
                                                       near=bem.NEAR_SKIP), args.warmup, args.steps)
        res[prec] = (times, A)
    import oracle
    om = oracle.OracleMesh(xyz, tri, 6)
    ref = om.entries(oracle.LAPLACE_SLP, oracle.P0, 0.0, idx, idx)
    nz = ref != 0
    err = {p: float(np.max(np.abs(res[p][1][nz] - ref[nz]) / np.abs(ref[nz]))) for p in res}
    n = idx.size * idx.size
    t64 = res[bem.FP64][0]
    line = {"metric": "weak-form entries/sec FP64 (dense P0 parity configuration)",
            "value": n / float(np.median(t64)), "unit": "entries/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": float(np.median(t64)) * 1e3, "higher_is_better": True,
            "scaling": "strong", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "Laplace single layer, P0, 6-point rule, icosphere level 3 (1280 triangles), all "
                                   "1,638,400 entries in one request (1,621,820 regular, vertex-sharing pairs 0)"},
            "seconds_min": min(t64), "fp32_entries_per_s": n / float(np.median(res[bem.FP32][0])),
            "max_rel_err_fp64": err[bem.FP64], "max_rel_err_fp32": err[bem.FP32], "regular_entries": int(nz.sum())}
    print(json.dumps(line))


def main():
    args = parse()
    if args.traffic_from:
        traffic_from(args)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the request server drives one device (a multi-GPU run would route "
              "blocks to independent per-GPU servers).", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.dense:
        dense_main(args)
        return
    if args.complete:
        complete_main(args)
        return
    if args.workload == "cylinder":
        cylinder_main(args)
        return
    if args.workload == "spheroid":
        spheroid_main(args)
        return
    if args.workload == "mix":
        mix_main(args)
        return
    if args.workload == "sphere3":
        sphere3_main(args)
        return
    from paper_1711_01897_amd import bem, inputs

    xyz, tri = inputs.icosphere(6)
    mesh = bem.mesh_create(xyz, tri, 6)
    print(f"[bench] mesh {tri.shape[0]} triangles / {xyz.shape[0]} vertices resident", file=sys.stderr, flush=True)

    dt, tot, sst, kst = timed(bem, mesh, bem.FP32, args.steps, args.warmup, args)
    print(f"[bench] fp32: {args.steps} steps in {dt:.3f} s, {tot['entries']} entries", file=sys.stderr, flush=True)
    roof, dom = roofline(kst)

    fp64 = None
    if not args.no_fp64:
        # the same protocol as the FP32 leg: warm-ups, then the timed steps
        dt64, tot64, sst64, kst64 = timed(bem, mesh, bem.FP64, args.steps, args.warmup, args)
        t64 = sorted(tot64["step_seconds"])
        fp64 = {"value": tot64["entries"] / dt64, "unit": "entries/s", "seconds_per_step": dt64 / args.steps,
                "step_seconds_median": t64[len(t64) // 2], "step_seconds_min": t64[0],
                "aca_entries_per_step": tot64["entries"] // args.steps,
                "aca_requests_per_step": tot64["requests"] // args.steps,
                "latency_p50_ms": sst64["latency_p50"] * 1e3, "latency_p99_ms": sst64["latency_p99"] * 1e3,
                "rank_sum": tot64["rank_sum"] // args.steps, "kernel_entries_per_s": kernel_entries_rate(kst64)}
        print(f"[bench] fp64: {args.steps} steps in {dt64:.3f} s", file=sys.stderr, flush=True)

    cpu = None
    worst = None
    cpu_h = None
    if not args.no_cpu_baseline:
        cpu, worst = cpu_baseline(bem, inputs, mesh, xyz, tri, args.cpu_seconds, step_ops(args))
        print(f"[bench] cpu baseline {cpu['value']:.3e} entries/s on {cpu['cores']} threads", file=sys.stderr,
              flush=True)
        if args.cpu_hmatrix_fraction > 0:
            cpu_h = cpu_hmatrix(inputs, xyz, tri, step_ops(args), args.cpu_hmatrix_fraction)
            cpu_h["speedup_over_fp32_step"] = cpu_h["extrapolated_seconds"] / (dt / args.steps)
            print(f"[bench] cpu H-matrix: {cpu_h['extrapolated_seconds']:.1f} s extrapolated "
                  f"(S = {cpu_h['speedup_over_fp32_step']:.0f})", file=sys.stderr, flush=True)

    value = tot["entries"] / dt
    line = {
        "metric": "weak-form entries/sec FP32 vs FP64 at stated rel err; p50/p99 ACA request latency",
        "value": value,
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": workload_name(args),
            "aca_entries_per_step": tot["entries"] // args.steps,
            "aca_requests_per_step": tot["requests"] // args.steps,
            "admissible_blocks_per_step": tot["blocks"] // args.steps,
            "mean_rank": tot["rank_sum"] / max(1, tot["blocks"]),
            "max_rank": tot["rank_max"],
            "rank_sum_per_step": tot["rank_sum"] // args.steps,
            "workers": args.workers,
            "blocks_per_worker": args.blocks_per_worker,
        },
        "latency_p50_ms": sst["latency_p50"] * 1e3,
        "latency_p99_ms": sst["latency_p99"] * 1e3,
        "fused_launch_batches": sst["batches"],
        "requests_per_batch": sst["requests"] / max(1, sst["batches"]),
        "assembly_seconds_per_step": tot["phases"],
        "step_seconds_median": sorted(tot["step_seconds"])[len(tot["step_seconds"]) // 2],
        "step_seconds_min": min(tot["step_seconds"]),
        "server_seconds_per_step": {"dispatch": sst["dispatch_seconds"] / args.steps,
                                    "dispatch_hip_calls": sst["dispatch_hip_seconds"] / args.steps,
                                    "complete": sst["complete_seconds"] / args.steps,
                                    "event_wait": sst["wait_seconds"] / args.steps,
                                    "entry_kernels": sst["kernel_seconds"] / args.steps},
        "request_latency_legs_us": {k: round(sst["mean_%s_seconds" % k] * 1e6, 1)
                                    for k in ("queue", "stage", "device", "complete")},
        "kernel_busy_fraction": sst["kernel_seconds"] / dt if dt > 0 else None,
        "fp64": fp64,
        "fp32_over_fp64": (value / fp64["value"]) if fp64 else None,
        "kernel_entries_per_s": kernel_entries_rate(kst),
        "max_rel_err_sampled": worst,
        "roofline": roof,
        "cpu_baseline": cpu,
        "cpu_hmatrix": cpu_h,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
