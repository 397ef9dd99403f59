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


def cpu_baseline(p, threads, per_thread):
    """Oracle gate bootstraps (blind rotation + extraction + key switch) at the
    workload's parameters on random key material (the work does not depend
    on the key values), `per_thread` bootstraps on each of `threads` threads."""
    import oracle
    import seeded_inputs as si
    rows = (p.k + 1) * p.l
    bsk = si.torus(5, 3, p.n * rows * (p.k + 1) * p.N, p.q)
    ksk = si.torus(5, 5, p.k * p.N * p.ks_t * (1 << p.ks_bits) * (p.n + 1), p.q)
    lwe = si.torus(5, 7, threads * per_thread * (p.n + 1), p.q).reshape(-1, p.n + 1)
    oracle.lib()
    t0 = time.perf_counter()
    oracle.parallel_map(lambda i: oracle.gate_bootstrap(p, bsk, ksk, lwe[i]), range(len(lwe)), threads)
    dt = time.perf_counter() - t0
    return {"value": len(lwe) / dt, "unit": "bootstraps/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(lwe)} oracle gate bootstraps (n={p.n}, N={p.N}, l={p.l}) on {threads} threads, "
                      f"{dt:.1f} s wall"}


def counter_traffic():
    """HBM bytes per 4096-ciphertext blind-rotation launch from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE scaled by what they
    read for a 256 MiB copy), or None when the kernel source has changed since
    the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "br_mfma_std_batch4096_counters.json")
    src = os.path.join(ROOT, "paper_2510_15413_amd", "csrc", "br_mfma.hip")
    try:
        with open(path) as f:
            prof = json.load(f)
        with open(src, "rb") as f:
            h = hashlib.sha256(f.read()).hexdigest()[:16]
    except OSError:
        return None
    if prof.get("source_sha256_16") != h:
        return None
    return prof


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
