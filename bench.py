"""Benchmark of the FHE-SQL oblivious-selection hot path on one MI355X.

One step = the standard 32-bit gate parameter workload (n=630, N=1024, l=3,
Bg=2^7, key switching 2^2 x 8): a 4096-row table of two uniform 8-bit
columns, scanned twice -- mask(col1 == c) with c the value of a seeded row,
and mask(col1 < c) with c uniform -- each followed by the masked select of
col2 (If-Then-Else(mask, col2, enc(0)) per bit).  That is 4096 x (15 + 8) +
4096 x (8 + 8) = 159,744 gate bootstraps and 8192 encrypted rows per step.
Keys and ciphertexts are generated on the device from seeded streams and are
resident in HBM before the timed region.

Reported: bootstraps/s of the whole step (the value), encrypted rows/s, the
plain scalar-integer kernel against the int8-MFMA kernel on one 4096-ciphertext
bootstrap batch, the blind-rotation kernel's achieved int8 TOP/s against the
MI355X dense int8 peak (timed per launch with HIP events inside the library),
and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TFHE bootstraps/s + encrypted rows/s (WHERE mask+select), MFMA vs plain"
INT8_PEAK_TOPS = 5000.0  # MI355X dense int8 MFMA, 5.0 POP/s
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def int8_ops_per_bootstrap(p):
    """Algorithmic int8 MFMA operations of one blind rotation:
    n steps x 2 * (k+1)N rows * (k+1)lN columns * limbs."""
    limbs = 4 if p.q == 32 else 8
    return 2.0 * (p.k + 1) * p.N * (p.k + 1) * p.l * p.N * limbs * p.n


def cpu_model():
    """CPU model name from /proc/cpuinfo (or the platform string)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(p, threads, per_thread, single=4):
    """Oracle gate bootstraps (blind rotation + extraction + key switch) at the
    workload's parameters on random key material (the work does not depend
    on the key values): `single` bootstraps on one thread, then `per_thread`
    bootstraps on each of `threads` threads (the process's CPU share, at most
    16).  value / cores describe the multi-threaded run."""
    import oracle
    import seeded_inputs as si
    rows = (p.k + 1) * p.l
    bsk = si.torus(5, 3, p.n * rows * (p.k + 1) * p.N, p.q)
    ksk = si.torus(5, 5, p.k * p.N * p.ks_t * (1 << p.ks_bits) * (p.n + 1), p.q)
    lwe = si.torus(5, 7, max(threads * per_thread, single) * (p.n + 1), p.q).reshape(-1, p.n + 1)
    oracle.lib()
    t0 = time.perf_counter()
    for i in range(single):
        oracle.gate_bootstrap(p, bsk, ksk, lwe[i])
    dt1 = time.perf_counter() - t0
    cnt = threads * per_thread
    t0 = time.perf_counter()
    oracle.parallel_map(lambda i: oracle.gate_bootstrap(p, bsk, ksk, lwe[i]), range(cnt), threads)
    dt = time.perf_counter() - t0
    return {"value": cnt / dt, "unit": "bootstraps/s", "cores": threads, "kind": "oracle",
            "single_core_value": single / dt1, "nproc": os.cpu_count(),
            "cpu_share": len(os.sched_getaffinity(0)), "cpu_model": cpu_model(),
            "sample": f"{single} oracle gate bootstraps (n={p.n}, N={p.N}, l={p.l}) on 1 thread in {dt1:.1f} s, "
                      f"then {cnt} on {threads} threads in {dt:.1f} s wall"}


def code_hash(path):
    """sha256[:16] of a kernel source with comments and blank lines removed,
    so that the committed counter summaries stay tied to the code alone."""
    import hashlib
    import re
    with open(path) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = [re.sub(r"//.*", "", ln).rstrip() for ln in text.splitlines()]
    return hashlib.sha256("\n".join(ln for ln in lines if ln.strip()).encode()).hexdigest()[:16]


def keyswitch_counters():
    """HBM rate of the 4096-ciphertext key switch from the committed counter
    summary, or None when keyswitch.hip has changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "keyswitch_std_batch4096_counters.json")
    src = os.path.join(ROOT, "paper_2510_15413_amd", "csrc", "keyswitch.hip")
    try:
        with open(path) as f:
            prof = json.load(f)
        h = code_hash(src)
    except OSError:
        return None
    if prof.get("code_sha256_16") != h:
        return None
    return {"kernel": prof["kernel"], "hbm_gb_per_s": round(prof["hbm_gbps"], 1), "hbm_peak_gb_per_s": 8000,
            "hbm_frac": round(prof["hbm_gbps"] / 8000, 4), "algorithmic_gb_per_s": round(prof["algorithmic_gbps"], 1),
            "ms_per_4096": round(prof["kernel_ms"], 3), "traffic_over_algorithmic": round(prof["traffic_over_algorithmic"], 2),
            "bound": "mfma (int8 limb products of the one-hot digits and the table, one staged table fragment per 4 MFMAs)"}


def counter_traffic():
    """HBM bytes per 4096-ciphertext blind-rotation launch from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE scaled by what they
    read for a 256 MiB copy), or None when the kernel source has changed since
    the counters were taken."""
    path = os.path.join(ROOT, "profiles", "br_mfma_std_batch4096_counters.json")
    src = os.path.join(ROOT, "paper_2510_15413_amd", "csrc", "br_mfma.hip")
    try:
        with open(path) as f:
            prof = json.load(f)
        h = code_hash(src)
    except OSError:
        return None
    if prof.get("code_sha256_16") != h:
        return None
    return prof


def param_desc(p):
    return f"{p.name} q={p.q} n={p.n} N={p.N} l={p.l} Bg=2^{p.bg_bits} ks 2^{p.ks_bits}x{p.ks_t}"


def batch16(args):
    """16 tables with log-uniform row counts in [100, 65536] and 16-bit
    columns, each with one predicate (==, <, BETWEEN) and the masked select of
    its second column, all tables' gates merged level by level and captured
    in one HIP graph; toy parameters by default, --params std for the
    standard gate set."""
    import torch
    import seeded_inputs as si
    import paper_2510_15413_amd as fs
    from paper_2510_15413_amd import client, autotune
    p = si.PARAMS[args.params]
    w = 16
    seed = si.DATA_SEED_BASE + 3
    rows_t, ops_t = si.uneven_tables(seed)
    s, S, bsk, ksk = fs.tfhe_keygen(p, si.KEY_SEED_BASE + 3)
    ctx = fs.Context(p, bsk, ksk)
    del bsk, ksk
    dev = torch.device("cuda")
    names = ["eq", "lt", "between"]
    queries, truths = [], []
    bs_total = 0
    for t, (rows, opi) in enumerate(zip(rows_t.tolist(), ops_t.tolist())):
        op = names[opi]
        col1, col2 = si.table(seed, rows, w, table_id=t)
        lits = si.uniform_ints(seed, si.TAG_LITERAL | (t << 32), 3, w)
        if op == "eq":
            a, b = int(col1[int(lits[0]) % rows]), None
        elif op == "lt":
            a, b = int(lits[1]), None
        else:
            a, b = sorted((int(lits[1]), int(lits[2])))
        enc = lambda vals, tag: client.encrypt_bits(  # noqa: E731
            p, seed, s, client.value_bits(torch.as_tensor(vals, dtype=torch.int64, device=dev), w), tag_hi=tag)
        q = dict(col=enc(col1.astype("int64"), 100 + 4 * t), sel_col=enc(col2.astype("int64"), 101 + 4 * t),
                 rows=rows, w=w, op=op, lit_a=enc([a], 102 + 4 * t)[0],
                 lit_b=enc([b], 103 + 4 * t)[0] if b is not None else None,
                 mask=torch.empty((rows, p.n + 1), dtype=torch.int32, device=dev),
                 sel_out=torch.empty((rows, w, p.n + 1), dtype=torch.int32, device=dev))
        queries.append(q)
        truth = (col1 == a) if op == "eq" else (col1 < a) if op == "lt" else ((col1 >= a) & (col1 <= b))
        truths.append(truth)
        bs_total += rows * ({"eq": 2 * w - 1, "lt": w, "between": 2 * w + 1}[op] + w)
    torch.cuda.synchronize()
    log(f"batch16: {int(rows_t.sum())} rows in 16 tables, {bs_total} bootstraps per run")

    def run():
        ctx.sql_scan_batch(queries, use_graph=True)
        torch.cuda.synchronize()

    tuned = None
    if args.autotune:
        tuned, _ = autotune.tune(ctx, f"batch16-{bs_total}", run, cache_path=None, log=log)
    for _ in range(args.warmup):
        run()
    ctx.timing_enable(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        run()
        log(f"batch16 run {i + 1}/{args.steps}: {time.perf_counter() - t0:.2f} s")
    wall = time.perf_counter() - t0
    # the graph's kernels are not event-timed; time one ungraphed run for the kernel split
    ctx.sql_scan_batch(queries, use_graph=False)
    torch.cuda.synchronize()
    br_n, br_ms, br_cts = ctx.timing_read("br")
    ctx.timing_enable(False)
    ok = all(bool((client.decrypt_bits(p, s, q["mask"]).cpu().numpy() == tr).all()) for q, tr in zip(queries, truths))
    ops_bs = int8_ops_per_bootstrap(p)
    ach = br_cts * ops_bs / (br_ms * 1e-3) / 1e12 if br_ms > 0 else 0.0
    res = {"workload": "batch16", "params": param_desc(p), "tables": len(queries),
           "rows": int(rows_t.sum()), "rows_per_table": rows_t.tolist(), "ops": [names[o] for o in ops_t.tolist()],
           "bootstraps_per_run": bs_total, "runs": args.steps, "seconds_per_run": round(wall / args.steps, 4),
           "bootstraps_per_s": round(bs_total * args.steps / wall, 1),
           "rows_per_s": round(int(rows_t.sum()) * args.steps / wall, 1), "hipgraph": True,
           "tuning": tuned, "decrypt_ok": ok,
           "ungraphed_kernel_split": {"br_launches": br_n, "br_ms": round(br_ms, 2),
                                      "br_achieved_int8_tops": round(ach, 1)}}
    ctx.close()
    print(json.dumps(res), flush=True)


def serve(args):
    """Open-loop Poisson arrivals of SELECT SUM(col2) WHERE col1 op c over a
    prefix of one resident table (8-bit columns; toy parameters by default,
    --params std for the standard gate set), prefix lengths log-uniform in
    [1e3, max_rows], op uniform over {==, <, >}."""
    import torch
    import seeded_inputs as si
    import paper_2510_15413_amd as fs
    from paper_2510_15413_amd import client, serve as srv
    p = si.PARAMS[args.params]
    w = 8
    seed = si.DATA_SEED_BASE + 5
    s, S, bsk, ksk = fs.tfhe_keygen(p, si.KEY_SEED_BASE + 5)
    ctx = fs.Context(p, bsk, ksk)
    del bsk, ksk
    dev = torch.device("cuda")
    R = args.max_rows
    col1, col2 = si.table(seed, R, w)
    t1 = torch.from_numpy(col1.astype("int64")).to(dev)
    t2 = torch.from_numpy(col2.astype("int64")).to(dev)
    c1 = torch.empty((R, w, p.n + 1), dtype=torch.int32, device=dev)
    c2 = torch.empty_like(c1)
    step = 1 << 16
    for r0 in range(0, R, step):  # encrypt in slices to bound temporaries
        r1 = min(R, r0 + step)
        c1[r0:r1] = client.encrypt_bits(p, seed, s, client.value_bits(t1[r0:r1], w), tag_hi=1, start=r0 * w)
        c2[r0:r1] = client.encrypt_bits(p, seed, s, client.value_bits(t2[r0:r1], w), tag_hi=2, start=r0 * w)
    torch.cuda.synchronize()
    log(f"serve: table of {R} rows encrypted")
    free, total = torch.cuda.mem_get_info()
    budget = int(free * 0.8) + (total - free) // 8
    results = []
    names = ["eq", "lt", "gt"]
    for li, lam in enumerate(float(x) for x in args.rates.split(",")):
        n = args.queries
        rows = si.log_uniform_int(seed + li, si.TAG_SHAPE, n, 1000, R).clip(1, R)
        ops = (si.uniform_ints(seed + li, si.TAG_SHAPE, n, 16, start=n) % 3).astype("int64")
        lits = si.uniform_ints(seed + li, si.TAG_LITERAL, n, w)
        arrivals = srv.poisson_arrivals(seed + li, n, lam)
        qs = []
        for i in range(n):
            op = names[int(ops[i])]
            lit = int(col1[int(lits[i]) % int(rows[i])]) if op == "eq" else int(lits[i])
            lt = client.encrypt_bits(p, seed, s, client.value_bits(torch.tensor([lit], device=dev), w)[0],
                                     tag_hi=1000 + 100 * li + i)
            qs.append(dict(col=c1, sum_col=c2, rows=int(rows[i]), w=w, op=op, lit_a=lt, lit=lit,
                           out=torch.empty((srv.sum_bits(w, int(rows[i])), p.n + 1), dtype=torch.int32,
                                           device=dev)))
        recs, stats = srv.run(ctx, qs, arrivals, budget, log=log)
        ok = True
        for q in qs:
            r = q["rows"]
            pred = {"eq": col1[:r] == q["lit"], "lt": col1[:r] < q["lit"], "gt": col1[:r] > q["lit"]}[q["op"]]
            got = int(client.bits_to_values(client.decrypt_bits(p, s, q["out"])[None, :]).item())
            ok &= got == int((col2[:r].astype("int64") * pred).sum())
        summ = srv.summarize(recs, stats)
        summ.update({"lambda": lam, "decrypt_ok": bool(ok), "mean_rows": float(rows.mean())})
        results.append(summ)
        log(f"serve lambda={lam}: p50 {summ['p50_s']:.2f} s p99 {summ['p99_s']:.2f} s "
            f"{summ['rows_per_s']:.0f} rows/s ok={ok}")
    ctx.close()
    print(json.dumps({"workload": "serve", "params": param_desc(p), "bits": w,
                      "table_rows": R, "hbm_budget_bytes": budget, "rates": results}), flush=True)


def pbs64(args):
    """64-bit programmable bootstrapping (n=750, N=2048, l=4, Bg=2^6, KS 2^3x6):
    32-bit columns as 8 radix blocks of 4 bits.  mask(col1 < c) by block-wise
    LUT comparison (4 levels) and the masked select of col2 (1 level) over
    --rows rows of the 65,536-row table (all of it with --rows 65536, in
    logged chunks of 4096 rows) measure throughput; the masked SUM mod 2^32 --
    a row tree whose every level is 8 sequential block levels -- is timed on
    the first --sum-rows selected rows."""
    import numpy as np
    import torch
    import seeded_inputs as si
    import paper_2510_15413_amd as fs
    p = si.PBS64
    nb = 8
    rows = min(args.rows, 65536)
    srows = min(args.sum_rows, rows)
    seed = si.DATA_SEED_BASE + 4
    t_setup = time.perf_counter()
    s, S, bsk, ksk = fs.tfhe_keygen(p, si.KEY_SEED_BASE + 4)
    ctx = fs.Context(p, bsk, ksk)
    del bsk, ksk
    dev = torch.device("cuda")
    col1, col2 = si.table(seed, rows, 32)
    c = int(si.uniform_ints(seed, si.TAG_LITERAL, 1, 32)[0])
    delta = 1 << 58

    def enc(vals, tag):
        v = torch.as_tensor(vals.astype("int64"), device=dev)
        bl = (v[:, None] >> (4 * torch.arange(nb, device=dev))) & 15
        mu = (bl.reshape(-1) * delta).contiguous()
        return fs.tfhe_lwe_encrypt(p, seed, s, mu, tag_hi=tag).reshape(len(vals), nb, p.n + 1)

    c1, c2 = enc(col1, 1), enc(col2, 2)
    lit = enc(np.array([c], dtype=np.uint64), 3)[0]
    mask = torch.empty((rows, p.n + 1), dtype=torch.int64, device=dev)
    sel = torch.empty((rows, nb, p.n + 1), dtype=torch.int64, device=dev)
    tot = torch.empty((nb, p.n + 1), dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    log(f"pbs64 setup {time.perf_counter() - t_setup:.1f} s")
    ctx.timing_enable(True)
    # rows are independent: large tables run in chunks of 4096 rows, each
    # logged, with the same output bits as one call
    chunk = 4096
    t_mask = t_sel = 0.0
    for r0 in range(0, rows, chunk):
        r1 = min(rows, r0 + chunk)
        t0 = time.perf_counter()
        ctx.sql_radix_mask_scan(c1[r0:r1], r1 - r0, nb, "lt", lit, mask[r0:r1])
        torch.cuda.synchronize()
        t_mask += time.perf_counter() - t0
        t0 = time.perf_counter()
        ctx.sql_radix_masked_select(mask[r0:r1], c2[r0:r1], r1 - r0, nb, sel[r0:r1])
        torch.cuda.synchronize()
        t_sel += time.perf_counter() - t0
        log(f"pbs64 rows {r0}..{r1}: mask {t_mask:.2f} s, select {t_sel:.2f} s so far")
    br_n, br_ms, br_cts = ctx.timing_read("br")
    t0 = time.perf_counter()
    ctx.sql_radix_sum(sel[:srows].contiguous(), srows, nb, tot)
    torch.cuda.synchronize()
    t_sum = time.perf_counter() - t0
    log(f"pbs64 sum of {srows} rows: {t_sum:.2f} s")
    ctx.timing_enable(False)

    def dec(cts):
        ph = fs.tfhe_lwe_phase(p, s, cts).cpu().numpy().view(np.uint64)
        return (((ph + np.uint64(delta // 2)) // np.uint64(delta)) % np.uint64(64)).astype(np.int64)
    m = dec(mask)
    tb = dec(tot)
    got = sum(int(b) << (4 * i) for i, b in enumerate(tb))
    pred = col1 < c
    ok_mask = bool((m == np.where(pred, 16, 0)).all())
    ok_sum = got == int((col2[:srows].astype(object) * pred[:srows]).sum()) % (1 << 32)
    ops = int8_ops_per_bootstrap(p)
    ms_pbs = rows * (2 * nb - 1) + rows * nb
    sum_pbs = (srows - 1) * (2 * nb - 1)
    sum_levels = nb * max(0, (srows - 1).bit_length())
    res = {"workload": "pbs64", "params": "q=64 n=750 N=2048 l=4 Bg=2^6 ks 2^3x6, 8 blocks x 4 bits",
           "rows_sampled": rows, "rows_full": 65536,
           "mask_select": {"pbs": ms_pbs, "seconds": round(t_mask + t_sel, 3),
                           "pbs_per_s": round(ms_pbs / (t_mask + t_sel), 1),
                           "rows_per_s": round(rows / (t_mask + t_sel), 2),
                           "br_launches": br_n, "br_ms": round(br_ms, 1),
                           "br_achieved_int8_tops": round(br_cts * ops / (br_ms * 1e-3) / 1e12, 1) if br_ms else 0},
           "sum": {"rows": srows, "pbs": sum_pbs, "sequential_levels": sum_levels, "seconds": round(t_sum, 2),
                   "seconds_per_level": round(t_sum / max(1, sum_levels), 3)},
           "ops_per_pbs": ops, "decrypt_ok": {"mask": ok_mask, "sum": bool(ok_sum)}}
    ctx.close()
    print(json.dumps(res), flush=True)


def where(args):
    """SELECT * FROM t WHERE age > 18 AND salary < 1000 (the expression-tree
    example of Section 4.3 B) over `rows` rows of two 16-bit columns at the
    standard gate parameters, the two literals encrypted by the client: one
    sql_expr_eval for the mask, then the masked select of both columns."""
    import torch
    import seeded_inputs as si
    import paper_2510_15413_amd as fs
    from paper_2510_15413_amd import client
    p = si.STD
    rows, w = args.rows, 16
    kseed, dseed = si.KEY_SEED_BASE + 2, si.DATA_SEED_BASE + 5
    dev = torch.device("cuda")
    t0 = time.perf_counter()
    s, S, bsk, ksk = fs.tfhe_keygen(p, kseed)
    ctx = fs.Context(p, bsk, ksk)
    del bsk, ksk
    age = si.uniform_ints(dseed, si.TAG_DATA, rows, 16) % 100
    sal = si.uniform_ints(dseed, si.TAG_DATA, rows, 16, start=rows) % 2000
    ta = torch.from_numpy(age.astype("int64")).to(dev)
    tsal = torch.from_numpy(sal.astype("int64")).to(dev)
    c_age = client.encrypt_bits(p, dseed, s, client.value_bits(ta, w), tag_hi=1)
    c_sal = client.encrypt_bits(p, dseed, s, client.value_bits(tsal, w), tag_hi=2)
    l_age = client.encrypt_bits(p, dseed, s, client.value_bits(torch.tensor([18], device=dev), w)[0], tag_hi=3)
    l_sal = client.encrypt_bits(p, dseed, s, client.value_bits(torch.tensor([1000], device=dev), w)[0], tag_hi=4)
    nodes = [{"kind": "column", "col": 0}, {"kind": "literal", "lit": 0}, {"kind": "cmp", "op": "gt", "a": 0, "b": 1},
             {"kind": "column", "col": 1}, {"kind": "literal", "lit": 1}, {"kind": "cmp", "op": "lt", "a": 3, "b": 4},
             {"kind": "and", "a": 2, "b": 5}]
    dt = ctx.dtype
    mask = torch.empty((rows, p.n + 1), dtype=dt, device=dev)
    sel_a = torch.empty((rows, w, p.n + 1), dtype=dt, device=dev)
    sel_s = torch.empty_like(sel_a)
    torch.cuda.synchronize()
    log(f"setup {time.perf_counter() - t0:.1f} s (keys + {rows}-row table on device)")

    def step():
        ctx.sql_expr_eval(nodes, [c_age, c_sal], rows, w, mask, lits=[l_age, l_sal])
        ctx.sql_masked_select(mask, c_age, rows, w, sel_a)
        ctx.sql_masked_select(mask, c_sal, rows, w, sel_s)

    bs_per_step = rows * (w + w + 1 + 2 * w)
    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    ctx.timing_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step()
        torch.cuda.synchronize()
        log(f"step {i + 1}/{args.steps}: {time.perf_counter() - t_start:.2f} s elapsed")
    wall = time.perf_counter() - t_start
    br_n, br_ms, br_cts = ctx.timing_read("br")
    ks_n, ks_ms, ks_cts = ctx.timing_read("ks")
    ctx.timing_enable(False)
    m = client.decrypt_bits(p, s, mask).cpu().numpy()
    va = client.bits_to_values(client.decrypt_bits(p, s, sel_a)).cpu().numpy()
    vs = client.bits_to_values(client.decrypt_bits(p, s, sel_s)).cpu().numpy()
    truth = (age > 18) & (sal < 1000)
    ok = bool((m == truth).all() and (va == age * truth).all() and (vs == sal * truth).all())
    ops_bs = int8_ops_per_bootstrap(p)
    achieved = br_cts * ops_bs / (br_ms * 1e-3) / 1e12 if br_ms > 0 else 0.0
    print(json.dumps({
        "workload": "where", "metric": METRIC, "value": round(bs_per_step * args.steps / wall, 1),
        "unit": "bootstraps/s", "steps": args.steps, "ms_per_step": round(1e3 * wall / args.steps, 2),
        "config": {"workload": f"std gate params; {rows} rows x two 16-bit columns; "
                               "SELECT * WHERE age > 18 AND salary < 1000 (encrypted literals)",
                   "rows": rows, "bits": w, "bootstraps_per_step": bs_per_step},
        "rows_per_s": round(rows * args.steps / wall, 1), "selectivity": round(float(truth.mean()), 4),
        "decrypt_ok": ok,
        "kernels": {"blind_rotation": {"launches": br_n, "ms": round(br_ms, 2), "cts": br_cts},
                    "key_switch": {"launches": ks_n, "ms": round(ks_ms, 2), "cts": ks_cts}},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 1), "peak": INT8_PEAK_TOPS, "unit": "TOP/s",
                     "frac": round(achieved / INT8_PEAK_TOPS, 4), "kernel": "br_mfma_kernel"},
    }), flush=True)


def kernel_only(p):
    import torch
    import seeded_inputs as si
    import paper_2510_15413_amd as fs
    s, S, bsk, ksk = fs.tfhe_keygen(p, si.KEY_SEED_BASE + 2)
    ctx = fs.Context(p, bsk, ksk)
    B = 4096
    raw = fs.tfhe_rng_fill(0xB0, 1, B * (p.n + 1) // 2 + 1)
    lwe = raw.view(torch.int32)[: B * (p.n + 1)].reshape(B, p.n + 1).contiguous()
    big = torch.empty((B, p.N + 1), dtype=torch.int32, device="cuda")
    out = torch.empty((B, p.n + 1), dtype=torch.int32, device="cuda")
    x = torch.ones(64 << 20, dtype=torch.int32, device="cuda")  # 256 MiB
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    ctx.timing_enable(True)
    ctx.tfhe_bootstrap_batch(lwe, big)
    ctx.tfhe_keyswitch_batch(big, out)
    y.copy_(x)
    torch.cuda.synchronize()
    n, ms, cts = ctx.timing_read("br")
    log(f"kernel-only: blind rotation of {B} in {ms:.2f} ms; 256 MiB copy done")
    print(json.dumps({"mode": "kernel-only", "br_ms": ms, "batch": B,
                      "achieved_tops": B * int8_ops_per_bootstrap(p) / (ms * 1e-3) / 1e12}))
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--rows", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-kernel comparison")
    ap.add_argument("--workload", default="std", choices=["std", "batch16", "serve", "pbs64", "where"],
                    help="std: the headline 4096-row scan; batch16: 16 uneven tables at toy "
                         "parameters in one level-batched hipGraph schedule")
    ap.add_argument("--autotune", action="store_true", help="batch16: tune the executor knobs first")
    ap.add_argument("--params", default="toy", choices=["toy", "std"],
                    help="batch16 and serve: TFHE parameter set")
    ap.add_argument("--rates", default="1,2,4,8,16,32,64", help="serve: Poisson rates (queries/s)")
    ap.add_argument("--queries", type=int, default=16, help="serve: queries per rate")
    ap.add_argument("--max-rows", type=int, default=1 << 20, help="serve: largest table prefix")
    ap.add_argument("--sum-rows", type=int, default=4, help="pbs64: rows in the timed SUM tree")
    ap.add_argument("--kernel-only", action="store_true",
                    help="profiling mode: one 4096-ciphertext MFMA blind rotation, one key switch and a "
                         "256 MiB device copy (the counter calibration), then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the hot path is single-GPU here.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import seeded_inputs as si
    import paper_2510_15413_amd as fs
    from paper_2510_15413_amd import client

    p = si.STD
    if args.kernel_only:
        return kernel_only(p)
    if args.workload == "batch16":
        return batch16(args)
    if args.workload == "serve":
        return serve(args)
    if args.workload == "pbs64":
        return pbs64(args)
    if args.workload == "where":
        return where(args)
    rows, w = args.rows, 8
    kseed, dseed = si.KEY_SEED_BASE + 2, si.DATA_SEED_BASE + 2
    dev = torch.device("cuda")
    torch.cuda.init()
    t0 = time.perf_counter()
    s, S, bsk, ksk = fs.tfhe_keygen(p, kseed)
    ctx = fs.Context(p, bsk, ksk)
    del bsk, ksk
    col1, col2 = si.table(dseed, rows, w)
    rstar = int(si.uniform_ints(dseed, si.TAG_LITERAL, 1, 32)[0] % rows)
    c_eq = int(col1[rstar])
    c_lt = int(si.uniform_ints(dseed, si.TAG_LITERAL, 1, w, start=1)[0])
    t1 = torch.from_numpy(col1.astype("int64")).to(dev)
    t2 = torch.from_numpy(col2.astype("int64")).to(dev)
    c1 = client.encrypt_bits(p, dseed, s, client.value_bits(t1, w), tag_hi=1)
    c2 = client.encrypt_bits(p, dseed, s, client.value_bits(t2, w), tag_hi=2)
    lit_eq = client.encrypt_bits(p, dseed, s, client.value_bits(torch.tensor([c_eq], device=dev), w)[0], tag_hi=3)
    lit_lt = client.encrypt_bits(p, dseed, s, client.value_bits(torch.tensor([c_lt], device=dev), w)[0], tag_hi=4)
    dt = ctx.dtype
    mask_eq = torch.empty((rows, p.n + 1), dtype=dt, device=dev)
    mask_lt = torch.empty_like(mask_eq)
    sel_eq = torch.empty((rows, w, p.n + 1), dtype=dt, device=dev)
    sel_lt = torch.empty_like(sel_eq)
    torch.cuda.synchronize()
    log(f"setup {time.perf_counter() - t0:.1f} s (keys + {rows}-row table on device)")

    def step():
        ctx.sql_mask_scan(c1, rows, w, "eq", lit_eq, mask_eq)
        ctx.sql_masked_select(mask_eq, c2, rows, w, sel_eq)
        ctx.sql_mask_scan(c1, rows, w, "lt", lit_lt, mask_lt)
        ctx.sql_masked_select(mask_lt, c2, rows, w, sel_lt)

    bs_per_step = rows * ((2 * w - 1) + w) + rows * (w + w)
    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    ctx.timing_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step()
        torch.cuda.synchronize()
        log(f"step {i + 1}/{args.steps}: {time.perf_counter() - t_start:.2f} s elapsed")
    wall = time.perf_counter() - t_start
    br_n, br_ms, br_cts = ctx.timing_read("br")
    ks_n, ks_ms, ks_cts = ctx.timing_read("ks")
    ctx.timing_enable(False)

    # decrypt check of the last step's masks and selected values
    m_eq = client.decrypt_bits(p, s, mask_eq).cpu().numpy()
    m_lt = client.decrypt_bits(p, s, mask_lt).cpu().numpy()
    v_eq = client.bits_to_values(client.decrypt_bits(p, s, sel_eq)).cpu().numpy()
    decrypt_ok = bool((m_eq == (col1 == c_eq)).all() and (m_lt == (col1 < c_lt)).all()
                      and (v_eq == (col2 * (col1 == c_eq))).all())

    ops_bs = int8_ops_per_bootstrap(p)
    achieved = br_cts * ops_bs / (br_ms * 1e-3) / 1e12 if br_ms > 0 else 0.0
    bs_per_s = bs_per_step * args.steps / wall
    res = {
        "metric": METRIC, "value": round(bs_per_s, 1), "unit": "bootstraps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * wall / args.steps, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic (seeded keys and uniform 8-bit columns generated on the device)",
        "config": {"workload": f"std gate params n=630 N=1024 l=3 Bg=2^7 ks 2^2x8; {rows} rows x two 8-bit "
                               f"columns; mask(col1 == c) + select(col2), mask(col1 < c) + select(col2)",
                   "rows": rows, "bits": w, "bootstraps_per_step": bs_per_step, "kernel": "mfma"},
        "rows_per_s": round(2 * rows * args.steps / wall, 1),
        "decrypt_ok": decrypt_ok,
        "kernels": {"blind_rotation": {"launches": br_n, "ms": round(br_ms, 2), "cts": br_cts},
                    "key_switch": {"launches": ks_n, "ms": round(ks_ms, 2), "cts": ks_cts}},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 1), "peak": INT8_PEAK_TOPS, "unit": "TOP/s",
                     "frac": round(achieved / INT8_PEAK_TOPS, 4), "traffic": None,
                     "kernel": "br_mfma_kernel", "ops_per_bootstrap": ops_bs},
    }

    prof = counter_traffic()
    if prof is not None:
        res["roofline"]["traffic"] = round(prof["hbm_bytes_per_launch"])
        res["roofline"]["traffic_launch"] = "4096-ciphertext launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)"
        res["roofline"]["algorithmic_bytes_per_launch"] = 4096 * (p.n + 1 + p.N + 1) * 4 + \
            p.n * 2 * p.l * 2 * 4 * 2 * p.N
        res["roofline"]["mfma_busy_frac_counter"] = round(prof["mfma_busy_frac"], 4)
    ksc = keyswitch_counters()
    if ksc is not None:
        res["key_switch_counters"] = ksc

    if not args.no_plain:
        B = 4096
        lwe = c1.reshape(-1, p.n + 1)[:B].contiguous()
        out_m = torch.empty((B, p.N + 1), dtype=dt, device=dev)
        out_p = torch.empty_like(out_m)
        times = {}
        for kind, out in (("mfma", out_m), ("plain", out_p)):
            ctx.set_kernel(kind)
            ctx.tfhe_bootstrap_batch(lwe, out)  # warm
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ctx.tfhe_bootstrap_batch(lwe, out)
            e1.record()
            torch.cuda.synchronize()
            times[kind] = e0.elapsed_time(e1) * 1e-3
            log(f"{kind} kernel: {B} bootstraps in {times[kind]:.3f} s")
        ctx.set_kernel("mfma")
        res["plain"] = {"batch": B, "mfma_bs_per_s": round(B / times["mfma"], 1),
                        "plain_bs_per_s": round(B / times["plain"], 1),
                        "mfma_over_plain": round(times["plain"] / times["mfma"], 2),
                        "identical_bits": bool(torch.equal(out_m, out_p))}

    if not args.no_cpu:
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        res["cpu_baseline"] = cpu_baseline(p, threads, 2)
        log(f"cpu baseline: {res['cpu_baseline']['sample']}")
    ctx.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
