"""Benchmark: RSA-2048 CRT decryptions per second on one MI355X.

One step = one CRT decryption of a batch of 16384 ciphertexts (seeded, uniform
in [0, n), one seeded RSA-2048 key, full-length d_p and d_q) resident in HBM:
the two 1024-bit half exponentiations in one launch, then the Garner launch.
Prints one JSON line (see the design doc for every field).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--window w]
  python bench.py --sweep-window      # one line per window width 1..6
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import random
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RSA-2048 CRT decrypts/sec on 1 MI355X (batched vs plain), p50/p99 latency"
# MI355X: 256 CUs x 64 lanes/clock x 2.4 GHz, the full per-lane VALU issue
# rate.  The rate of v_mad_u64_u32 (32x32->64 multiply-add) itself is
# measured on the device (rns_probe_alu) and reported beside it.
PEAK_MUL_PER_S = 256 * 64 * 2.4e9
# MI355X dense int8 matrix-core peak (v_mfma_i32_16x16x64_i8): 5.0 POP/s.
PEAK_I8_OPS_PER_S = 5.0e15
ENGINE_NAMES = {1: "channel", 2: "matrix"}
KERNEL_SOURCES = ["paper_1305_3699_amd/csrc/kernels_impl.hpp", "paper_1305_3699_amd/csrc/arith.hpp",
                  "paper_1305_3699_amd/csrc/kernel_configs.inc", "paper_1305_3699_amd/csrc/kernels_mfma.hpp",
                  "paper_1305_3699_amd/csrc/mfma_layout.hpp", "paper_1305_3699_amd/csrc/kernel_configs_mfma.inc",
                  "paper_1305_3699_amd/build.py"]
KERNELS = ("modexp_kernel", "modexp_mfma_kernel", "garner_kernel", "montmul_kernel")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def mm_count(exp: int, exp_bits: int, w: int, sliding: bool = True) -> int:
    """RNS Montgomery products of one exponentiation as the kernels schedule
    them.  sliding (matrix-core kernel, shared exponent): entry, x^2 and the
    odd powers up to x^(2^w - 1), then per sliding window after the first its
    squarings and one multiplication, one squaring per zero bit between
    windows, exit.  Fixed (channel kernel): entry, 2^w - 2 table products, w
    squarings per digit after the leading non-zero one plus one multiply per
    non-zero digit, exit."""
    if sliding:
        n = 2 + ((1 << (w - 1)) if w > 1 else 0)
        i = exp.bit_length() - 1
        first = True
        while i >= 0:
            if not (exp >> i) & 1:
                n += 1
                i -= 1
                continue
            lo = max(i - w + 1, 0)
            while not (exp >> lo) & 1:
                lo += 1
            if not first:
                n += (i - lo + 1) + 1
            first = False
            i = lo - 1
        return n
    nd = (exp_bits + w - 1) // w
    digits = [(exp >> (w * (nd - 1 - i))) & ((1 << w) - 1) for i in range(nd)]
    n = 1 + (1 << w) - 2 + 1
    started = False
    for d in digits:
        if not started:
            started = d != 0
            continue
        n += w + (1 if d else 0)
    return n


def wide_muls_per_mm(k: int) -> int:
    """Algorithmic 32x32->64 products of one RNS Montgomery product: the two
    base extensions (k(k+1) each) and seven per-channel products per channel."""
    return 2 * k * (k + 1) + 7 * k


def kernel_shape(info: dict) -> tuple:
    """Template arguments of the exponentiation kernel that serves info."""
    if info["engine"] != 2:
        return (info["k"], info["waves"])
    import re
    txt = open(os.path.join(ROOT, "paper_1305_3699_amd/csrc/kernel_configs_mfma.inc")).read()
    for m in re.finditer(r"RNSRSA_MSHAPE\((\d+),\s*(\d+),\s*(\d+),\s*(\d+)\)", txt):
        k, w, mt, nt = (int(v) for v in m.groups())
        if k == info["k"] and w == info["waves"] and 16 * nt == info["group"]:
            return (k, w, mt, nt)
    return (info["k"], info["waves"])


def probe_alu_rate(op: int):
    """Measured lane-ops/s of a wide multiply form (0: v_mad_u64_u32, 1:
    v_mad_i64_i32) on the current GPU, or None if the probe fails."""
    import ctypes

    from paper_1305_3699_amd import rnsrsa
    v = ctypes.c_double(0.0)
    return v.value if rnsrsa.lib().rns_probe_alu(op, ctypes.byref(v), None) == 0 else None


def i8_macs_per_mm(k: int) -> int:
    """Algorithmic int8 products of the two base extensions of one RNS
    Montgomery product on the matrix cores: k(k+1) residue products each
    (k inputs, k+1 outputs with the redundant channel), 16 byte products per
    32 x 32-bit residue product."""
    return 2 * 16 * k * (k + 1)


def cpu_threads() -> int:
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, min(n, 16))


def load_traffic(kernel_name: str):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except ValueError:
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash() or kernel_name not in rec.get("kernels", {}):
        return None
    return rec["kernels"][kernel_name].get("bytes_per_launch")


def ingest_counters(fetch_csv: str, write_csv: str, calib_mb: int) -> dict:
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch)
    into HBM bytes per launch of each kernel, scaled so that the calibration
    kernel (an elementwise copy reading and writing calib_mb MiB) reads exactly
    calib_mb MiB and writes calib_mb MiB; writes profiles/traffic.json."""
    import csv

    def per_kernel(path):
        rows = list(csv.DictReader(open(path)))
        vals = {}
        for r in rows:
            vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return vals

    f, w = per_kernel(fetch_csv), per_kernel(write_csv)
    known_kib = calib_mb * 1024.0
    calib = [v for name, vs in f.items() if "elementwise" in name for v in vs]
    fetch_scale = known_kib / max(calib)
    calib_w = [v for name, vs in w.items() if "elementwise" in name for v in vs]
    write_scale = known_kib / max(calib_w)
    out = {"kernel_source_hash": kernel_source_hash(), "fetch_scale": round(fetch_scale, 4),
           "write_scale": round(write_scale, 4), "calibration": "elementwise copy of %d MiB" % calib_mb,
           "kernels": {}}
    for name in f:
        short = name.split("(")[0].replace("void ", "").replace("rnsrsa::", "")
        base = short.split("<")[0]
        if base not in KERNELS:
            continue
        fk = statistics.mean(f[name]) * fetch_scale
        wk = statistics.mean(w.get(name, [0.0])) * write_scale
        out["kernels"][base] = {"instance": short, "fetch_kib": round(fk, 1), "write_kib": round(wk, 1),
                                "bytes_per_launch": int(round((fk + wk) * 1024))}
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def draw_keys(args) -> dict:
    """Every key of the run, drawn before the first GPU call (the mixed and
    served workloads' keys come from gen/keys.json; a process that has used
    the GPU must not fork a key-generation pool)."""
    import gen
    keys = {"c2": gen.rsa_key(2048, seed=gen.config_seed(2, 1))}
    if args.mixed_steps > 0:
        specs, ops = gen.mixed_batch_spec()
        keys["c4"] = (gen.rsa_keys(specs), ops)
    if args.served_default or args.served:
        keys["c5"] = gen.rsa_keys(gen.served_keys(per_size=64))
    return keys


def run(args, key, ref=None) -> dict:
    """The timed step on the C2 workload.  ref: the oracle's outputs for the
    batch, if already computed (then compared with, not timed again)."""
    import numpy as np
    import torch

    import gen
    from paper_1305_3699_amd import RsaKey

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs the GPU")
    torch.cuda.set_device(0)
    opts = {"window": args.window, "engine": args.engine, "group": args.group, "unscaled": args.unscaled}
    if args.waves:
        opts.update(k=33, waves=args.waves)
    rk = RsaKey(key.n, key.e, key.d, key.p, key.q, key.dp, key.dq, key.qinv, **opts)
    info = rk.info(1)
    B = args.batch
    c_int = gen.uniform_below(key.n, B, seed=gen.config_seed(2, 2))
    c_np = gen.to_limbs(c_int, 64)
    c = torch.from_numpy(c_np.view(np.int32)).cuda()
    half = rk.half_limbs
    mpq = torch.empty((B, 2 * half), dtype=torch.int32, device="cuda")
    m = torch.empty((B, 64), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    if args.calib_copy_mb:
        # a plain streaming kernel of known traffic (reads and writes N MiB) for
        # scaling hardware byte counters; runs before and outside the timed region
        n = args.calib_copy_mb * (1 << 20) // 4
        src = torch.zeros(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.add(src, 1, out=dst)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        rk.crt_halves(c, out=mpq)
        rk.crt_combine(mpq, out=m)
    torch.cuda.synchronize()

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
            torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b, d in evs:
        a.record(stream)
        rk.crt_halves(c, out=mpq)
        b.record(stream)
        rk.crt_combine(mpq, out=m)
        d.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    step_ms = [a.elapsed_time(d) for a, b, d in evs]
    modexp_ms = [a.elapsed_time(b) for a, b, d in evs]
    garner_ms = [b.elapsed_time(d) for a, b, d in evs]
    wall = t1 - t0
    value = B * args.steps / wall

    k = info["k"]
    sliding = info["engine"] == 2
    mms = (mm_count(key.dp, 32 * half, info["window"], sliding)
           + mm_count(key.dq, 32 * half, info["window"], sliding))
    muls_per_launch = B * mms * wide_muls_per_mm(k)
    mean_modexp_s = statistics.mean(modexp_ms) / 1e3
    achieved = muls_per_launch / mean_modexp_s

    kbase = "modexp_mfma_kernel" if info["engine"] == 2 else "modexp_kernel"
    kname = "%s<%s>" % (kbase, ",".join(map(str, kernel_shape(info))))
    valu = {
        "achieved": round(achieved / 1e12, 4),
        "peak": round(PEAK_MUL_PER_S / 1e12, 4),
        "unit": "Tmul/s",
        "frac": round(achieved / PEAK_MUL_PER_S, 4),
        "work_per_launch": muls_per_launch,
    }
    mad = probe_alu_rate(0)
    if mad:
        valu["peak_measured"] = round(mad / 1e12, 4)
        valu["frac_measured"] = round(achieved / mad, 4)
        valu["measured"] = "v_mad_u64_u32 lane-ops/s on this GPU (rns_probe_alu)"
    if info["engine"] == 2:
        ops = 2 * B * mms * i8_macs_per_mm(k)
        roofline = {"bound": "mfma", "kernel": kname,
                    "achieved": round(ops / mean_modexp_s / 1e12, 2), "peak": PEAK_I8_OPS_PER_S / 1e12,
                    "unit": "TOP/s", "frac": round(ops / mean_modexp_s / PEAK_I8_OPS_PER_S, 4),
                    "traffic": load_traffic(kbase), "work_per_launch": ops, "mm_per_decrypt": mms,
                    "what": "int8 ops of the two base extensions (2 x 16 k(k+1) MACs per RNS product)",
                    "wide_mul_equiv": valu}
    else:
        roofline = {"bound": "alu", "kernel": kname, **valu, "traffic": load_traffic(kbase),
                    "mm_per_decrypt": mms,
                    "what": "32x32->64 products W(k) = 2k(k+1) + 7k per RNS product vs full-rate VALU issue"}
    sq = sorted(step_ms)
    p50 = statistics.median(sq)
    p99 = sq[min(len(sq) - 1, int(round(0.99 * (len(sq) - 1))))]
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "decrypts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded RSA-2048 key, ciphertexts uniform in [0,n))",
        "config": {
            "workload": "RSA-2048 CRT decryption of %d ciphertexts per step, full-length d_p/d_q, "
                        "both 1024-bit halves in one launch, then Garner" % B,
            "form": "plain",
            "batch": B,
            "key_bits": 2048,
            "k": k,
            "waves": info["waves"],
            "window": info["window"],
            "engine": ENGINE_NAMES[info["engine"]],
            "group": info["group"],
            "scaled_b": bool(info["scaled"]),
        },
        "latency_ms": {"p50": round(p50, 4), "p99": round(p99, 4), "what": "one step (batch of %d)" % B},
        "modexps_per_s": round(2 * value, 1),
        "kernels_ms": {"modexp_crt_halves": round(statistics.mean(modexp_ms), 4),
                       "garner": round(statistics.mean(garner_ms), 4)},
        "roofline": roofline,
        "cpu_baseline": None,
    }
    got_all = m.cpu().numpy().view(np.uint32)
    if ref is not None:
        out["matches_oracle"] = bool(np.array_equal(ref, got_all))
    if args.cpu_sample > 0:
        import oracle
        ns = min(args.cpu_sample, B)
        threads = cpu_threads()
        sample = c_np[:ns]
        t2 = time.perf_counter()
        ref_s = oracle.rsa_crt_batch(sample, key.p, key.q, key.dp, key.dq, key.qinv, nthreads=threads)
        t3 = time.perf_counter()
        got = got_all[:ns]
        out["cpu_baseline"] = {
            "value": round(ns / (t3 - t2), 2),
            "unit": "decrypts/s",
            "cores": threads,
            "kind": "oracle",
            "sample": "first %d of the %d ciphertexts, the oracle's schoolbook CRT/Garner path, %.1f s wall"
                      % (ns, B, t3 - t2),
            "matches_gpu": bool(np.array_equal(ref_s, got)),
        }
        if ns == B:
            ref = ref_s
        # the correctness definition itself, c^d mod n, on a bounded sample
        npl = min(max(ns // 16, 1), B)
        t4 = time.perf_counter()
        refp = oracle.modexp_batch(c_np[:npl], np.array(gen.to_limbs(key.d, 64)[0]), np.array(gen.to_limbs(key.n, 64)[0]),
                                   nthreads=threads)
        t5 = time.perf_counter()
        out["cpu_baseline"]["plain"] = {
            "value": round(npl / (t5 - t4), 2), "unit": "decrypts/s",
            "sample": "first %d ciphertexts, the oracle's c^d mod n (schoolbook, no CRT), %.1f s wall" % (npl, t5 - t4),
            "matches_gpu": bool(np.array_equal(refp, got[:npl])),
        }
    return out, ref


def run_mixed(args, keys, ops) -> dict:
    """Batched vs plain on the mixed-size workload: 64 seeded keys over
    1024/2048/3072/4096 bits, lognormal per-key counts (median 128), half
    encryptions and half CRT decryptions.  plain = one rsa_encrypt /
    rsa_decrypt call per (key, op) in sequence on one stream; batched = one
    RsaBatch run (one grouped launch per kernel shape, hipGraph).  After the
    timed runs every batched output is compared with the oracle (all host
    threads, outside the timed region)."""
    import numpy as np
    import torch

    import gen
    import oracle
    from paper_1305_3699_amd import OP_DECRYPT, OP_ENCRYPT, RsaBatch, RsaKey

    rks = [RsaKey(k.n, k.e, k.d, k.p, k.q, k.dp, k.dq, k.qinv) for k in keys]
    items = []
    for o in ops:
        k = keys[o.key_index]
        vals = gen.uniform_below(k.n, o.count, seed=o.msg_seed)
        xl = gen.to_limbs(vals, o.bits // 32)
        inp = torch.from_numpy(xl.view(np.int32)).cuda()
        items.append((o, rks[o.key_index], inp, torch.empty_like(inp), torch.empty_like(inp), xl))
    n_ops = sum(o.count for o in ops)

    def plain_run():
        for o, rk, inp, out_p, _, _ in items:
            if o.kind == "encrypt":
                rk.encrypt(inp, out=out_p)
            else:
                rk.decrypt(inp, use_crt=True, out=out_p)

    t0 = time.perf_counter()
    batch = RsaBatch([(rk, OP_ENCRYPT if o.kind == "encrypt" else OP_DECRYPT, inp, out_b)
                      for o, rk, inp, _, out_b, _ in items], autotune=True, use_graph=True)
    create_s = time.perf_counter() - t0
    res = {}
    for name, fn in (("plain", plain_run), ("batched", batch.run)):
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(args.mixed_steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        ms.sort()
        res[name] = {"ops_per_s": round(n_ops / (statistics.mean(ms) / 1e3), 1),
                     "ms_p50": round(statistics.median(ms), 3), "ms_p99": round(ms[-1], 3)}
    same = all(torch.equal(out_p, out_b) for _, _, _, out_p, out_b, _ in items)
    info = batch.info
    classes = batch.classes
    batch.close()
    threads = cpu_threads()
    t0 = time.perf_counter()
    matches = True
    for o, rk, inp, _, out_b, xl in items:
        k = keys[o.key_index]
        got = out_b.cpu().numpy().view(np.uint32)
        if o.kind == "encrypt":
            want = oracle.modexp_batch(xl, gen.to_limbs(k.e, 1)[0], gen.to_limbs(k.n, o.bits // 32)[0],
                                       nthreads=threads)
        else:
            want = oracle.rsa_crt_batch(xl, k.p, k.q, k.dp, k.dq, k.qinv, nthreads=threads)
        matches = matches and bool(np.array_equal(got, want))
    oracle_s = time.perf_counter() - t0
    return {
        "workload": "64 keys (16 each of 1024/2048/3072/4096 bits), per-key counts lognormal(median 128, "
                    "sigma 1, cap 8192), each message encrypt or CRT-decrypt with p = 0.5",
        "ops": n_ops,
        "decrypts": sum(o.count for o in ops if o.kind == "decrypt"),
        "plain": res["plain"],
        "batched": res["batched"],
        "speedup": round(res["batched"]["ops_per_s"] / res["plain"]["ops_per_s"], 2),
        "batched_matches_plain": bool(same),
        "matches_oracle": matches,
        "oracle_check": "every output of the batched run vs the oracle (%d host threads, %.1f s)" % (threads, oracle_s),
        "launches_per_run": {"batched": info["launches"] + info["garner_launches"],
                             "plain": len(items) + sum(1 for o in ops if o.kind == "decrypt")},
        "graph": True,
        "autotuned": [{key: c[key] for key in ("k", "waves", "group", "exp_bits", "window", "window_offset", "jobs",
                                               "launch_ms")} for c in classes],
        "tuning_launches": info["tuning_launches"],
        "create_s": round(create_s, 2),
        "workspace_mb": round(info["workspace_bytes"] / 2 ** 20, 1),
    }


def run_served(args, keys) -> dict:
    """Served form: 256 resident keys (64 each of 2048/1024/3072/4096 bits),
    open-loop Poisson arrivals at each rate for warm-up + duration seconds,
    key size 40/30/20/10%, 70% CRT decryptions, 64 GiB admission budget.
    Latency = completion - arrival on the host clock; requests arriving during
    the warm-up are excluded.  A sample of each run is checked against the
    oracle."""
    import numpy as np

    import gen
    import oracle
    from paper_1305_3699_amd import RsaKey, RsaServer

    per = 64
    rks = [RsaKey(k.n, k.e, k.d, k.p, k.q, k.dp, k.dq, k.qinv) for k in keys]
    limbs = [k.n.bit_length() // 32 for k in keys]
    out = {"keys": len(keys), "budget_gib": 64,
           "max_inflight": args.served_inflight, "warmup_s": args.served_warmup,
           "duration_s": args.served_duration, "runs": []}
    for rate in args.served_rates:
        total = args.served_warmup + args.served_duration
        arrival, kidx, kind, seeds = gen.served_trace(rate, total, per_size=per, seed_offset=int(rate) % 1000)
        n = arrival.size
        msgs = np.zeros((n, 128), np.uint32)
        for i in range(n):
            L = limbs[kidx[i]]
            msgs[i, :L] = gen.to_limbs(gen.uniform_below_fast(keys[kidx[i]].n, int(seeds[i])), L)[0]
        for cap in args.served_max_ops:
            srv = RsaServer(rks, hbm_budget=64 << 30, max_inflight=args.served_inflight, max_dispatch_ops=cap)
            res, lat, st = srv.replay(kidx, kind, arrival, msgs)
            srv.close()
            sel = arrival >= args.served_warmup
            lw = np.sort(lat[sel])
            done_t = arrival + lat
            in_window = (done_t >= args.served_warmup) & (done_t < total)
            ok = True
            for i in random.Random(int(rate)).sample(range(n), min(64, n)):
                k = keys[kidx[i]]
                L = limbs[kidx[i]]
                x = np.ascontiguousarray(msgs[i:i + 1, :L])
                want = (oracle.modexp_batch(x, gen.to_limbs(k.e, 1)[0], gen.to_limbs(k.n, L)[0]) if kind[i] == 0
                        else oracle.rsa_crt_batch(x, k.p, k.q, k.dp, k.dq, k.qinv))
                ok = ok and bool(np.array_equal(res[i:i + 1, :L], want))
            out["runs"].append({
                "offered_req_per_s": rate,
                "max_dispatch_ops": cap or 16384,
                "requests": int(sel.sum()),
                "completed_per_s": round(float(in_window.sum()) / args.served_duration, 1),
                "latency_ms": {"p50": round(float(lw[(lw.size - 1) // 2]) * 1e3, 3),
                               "p99": round(float(lw[min(lw.size - 1, int(0.99 * (lw.size - 1) + 0.5))]) * 1e3, 3),
                               "max": round(float(lw[-1]) * 1e3, 3)},
                "dispatches": st["dispatches"],
                "mean_dispatch_requests": round(st["mean_dispatch_ops"], 1),
                "peak_inflight": st["peak_inflight"],
                "peak_inflight_mb": round(st["peak_inflight_bytes"] / 2 ** 20, 1),
                "sample_matches_oracle": ok,
            })
            print("served rate %g: %s" % (rate, json.dumps(out["runs"][-1])), file=sys.stderr, flush=True)
    return out


def run_modmul_sweep(args) -> list:
    """RNS modular multiplications per millisecond against the number of
    operands in flight (the shape of the paper's Fig. 1: 3072-bit modular
    multiplication over 128 32-bit channels, throughput vs blocks; and its
    note that doubling the channels reaches 8192-bit products).  Two forms:
    the standalone product (rns_mont_mul_batch, one launch of B independent
    products on residue vectors) and the products inside an exponentiation by
    an exponent as long as the modulus (rns_modexp_batch, counted from the
    exponent as the kernel schedules them).  3072 bits on k = 97 (the smallest
    base for that modulus) and k = 129 (the closest to the paper's 128
    channels); 8192 bits on k = 257 (256 + 1 channels)."""
    import numpy as np
    import torch

    import gen
    from paper_1305_3699_amd import RnsContext

    lines = []
    for bits, k in ((3072, 97), (3072, 129), (8192, 257)):
        L = bits // 32
        rng = random.Random(gen.config_seed(6, 1) if bits == 3072 else gen.config_seed(6, bits))
        N = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
        e = gen.random_exponent(bits, seed=gen.config_seed(6, 3) if bits == 3072 else gen.config_seed(6, bits + 3))
        el = torch.from_numpy(gen.to_limbs(e, L)[0].view(np.int32)).cuda()
        ctx = RnsContext(N, L, k=k, window=6)
        info = ctx.info
        primes = torch.tensor(ctx.primes + [0], dtype=torch.int64, device="cuda")
        mm_exp = mm_count(e, bits, info["window"], sliding=info["engine"] == 2)
        rows = []
        batches = [B for B in args.modmul_batches if bits == 3072 or B <= 16384]
        for B in batches:
            # standalone product: residues drawn below each channel modulus
            g = torch.Generator(device="cuda").manual_seed(B)
            def residues():
                r = torch.randint(0, 1 << 32, (2 * k + 1, B), dtype=torch.int64, device="cuda", generator=g)
                m = primes[:, None]
                r = torch.where(m > 0, r % torch.where(m > 0, m, 1), r)
                return torch.where(r >= 1 << 31, r - (1 << 32), r).to(torch.int32).contiguous()
            x, y = residues(), residues()
            out = torch.empty_like(x)

            def timed(fn, reps):
                for _ in range(2):
                    fn()
                torch.cuda.synchronize()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                for _ in range(reps):
                    fn()
                b.record()
                torch.cuda.synchronize()
                return a.elapsed_time(b) / reps

            ms_mm = timed(lambda: ctx.mont_mul(x, y, out=out), 20)
            bases = torch.from_numpy(gen.to_limbs([rng.getrandbits(bits - 1) for _ in range(min(B, 64))], L)
                                     .view(np.int32)).cuda().repeat((B + 63) // 64, 1)[:B].contiguous()
            res = torch.empty_like(bases)
            ms_exp = timed(lambda: ctx.modexp(bases, el, out=res), 2 if B >= 4096 else 5)
            rows.append({"operands": B, "standalone_per_ms": round(B / ms_mm, 1),
                         "in_exponentiation_per_ms": round(B * mm_exp / ms_exp, 1),
                         "standalone_ms": round(ms_mm, 4), "exponentiation_ms": round(ms_exp, 3)})
            print("modmul k=%d %s" % (k, json.dumps(rows[-1])), file=sys.stderr, flush=True)
        lines.append({"metric": "%d-bit RNS modular multiplications per ms vs operands in flight" % bits,
                      "bits": bits, "k": k, "engine": {1: "channel", 2: "matrix"}[info["engine"]],
                      "standalone_engine": {1: "channel", 2: "matrix"}[info["engine"]], "window": info["window"],
                      "products_per_exponentiation": mm_exp, "rows": rows})
    return lines


def run_keygen(args) -> dict:
    """The primality steps of key generation on 1024-bit candidates (the
    primes of an RSA-2048 key; Sec. 4.3): trial division by the first 10,000
    primes over a batch of seeded odd candidates (one launch, HIP events on
    its stream), then Miller-Rabin with 5 random bases (FIPS 186-4's count
    for 1024-bit primes) over the candidates that survive it (wall clock of
    the synchronous call: per-candidate contexts built on the host, grouped
    launches, read-backs).  The oracle runs the same steps on a CPU sample."""
    import numpy as np
    import torch

    import gen
    from oracle import primality
    from paper_1305_3699_amd import miller_rabin, trial_division

    rng = random.Random(gen.config_seed(9, 1))
    n = args.keygen_candidates
    cands = [rng.getrandbits(1024) | (3 << 1022) | 1 for _ in range(n)]
    cl = torch.from_numpy(gen.to_limbs(cands, 32).view(np.int32)).cuda()
    stream = torch.cuda.current_stream()
    flags = trial_division(cl, stream=stream)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(5):
        trial_division(cl, out=flags, stream=stream)
    b.record(stream)
    torch.cuda.synchronize()
    td_ms = a.elapsed_time(b) / 5
    keep = [c for c, f in zip(cands, flags.cpu().numpy()) if f]
    m = min(args.keygen_mr, len(keep))
    mr_c = keep[:m]
    brng = random.Random(gen.config_seed(9, 2))
    bases = [[brng.randrange(2, c - 1) for _ in range(5)] for c in mr_c]
    cl_mr, bl_mr = gen.to_limbs(mr_c, 32), np.stack([gen.to_limbs(x, 32) for x in bases])
    miller_rabin(cl_mr[:4], bl_mr[:4])                     # warm-up (kernels loaded, pools grown)
    t0 = time.perf_counter()
    verdict = miller_rabin(cl_mr, bl_mr)
    mr_s = time.perf_counter() - t0
    # oracle on a CPU sample of each step
    pr = primality.small_primes(10000)
    ns = min(2000, n)
    t0 = time.perf_counter()
    td_cpu = [primality.trial_division(c, primes=pr) for c in cands[:ns]]
    td_cpu_s = time.perf_counter() - t0
    nm = min(32, m)
    t0 = time.perf_counter()
    mr_cpu = [primality.miller_rabin(c, bs) for c, bs in zip(mr_c[:nm], bases[:nm])]
    mr_cpu_s = time.perf_counter() - t0
    # whole keys: rsa_keygen on seeded streams of 2500 1024-bit candidates per prime
    from paper_1305_3699_amd import keygen
    kt, nkeys = [], args.keygen_keys
    for kk in range(nkeys):
        krng = random.Random(gen.config_seed(9, 10 + kk))
        streams = []
        for _ in range(2):
            cs = [krng.getrandbits(1024) | (3 << 1022) | 1 for _ in range(2500)]
            bs = np.stack([gen.to_limbs([krng.randrange(2, c - 1) for _ in range(5)], 32) for c in cs])
            streams += [gen.to_limbs(cs, 32), bs]
        t0 = time.perf_counter()
        key = keygen(*streams, e=65537)
        kt.append(time.perf_counter() - t0)
        key.close()
    t0 = time.perf_counter()
    gen.rsa_key(2048, seed=gen.config_seed(9, 99))
    host_key_s = time.perf_counter() - t0
    return {"metric": "1024-bit prime candidates per second, trial division (10,000 primes) and Miller-Rabin (5 bases)",
            "rsa2048_keygen": {"keys": nkeys, "s_per_key": round(statistics.mean(kt), 4),
                               "s_per_key_max": round(max(kt), 4),
                               "host_generator_s_per_key": round(host_key_s, 3),
                               "what": "rsa_keygen on two seeded streams of 2500 candidates with 5 bases each "
                                       "(trial division, Miller-Rabin, Arazi's d in RNS, key load); host: the "
                                       "seeded pure-Python generator (40 rounds), one key"},
            "data": "synthetic", "candidates": n, "survive_trial_division": len(keep),
            "trial_division": {"ms": round(td_ms, 4), "candidates_per_s": round(n / td_ms * 1e3, 1)},
            "miller_rabin": {"candidates": m, "probable_primes": int(verdict.sum()), "s": round(mr_s, 4),
                             "candidates_per_s": round(m / mr_s, 1)},
            "cpu_oracle": {"trial_division_per_s": round(ns / td_cpu_s, 1),
                           "miller_rabin_per_s": round(nm / mr_cpu_s, 1), "cores": 1,
                           "sample": "%d and %d of the same candidates" % (ns, nm),
                           "matches_gpu": [bool(f) for f in flags.cpu().numpy()[:ns]] == td_cpu
                           and [bool(v) for v in verdict[:nm]] == mr_cpu}}


def run_configs(args) -> list:
    """The other measured configurations, one line each: the RSA-1024 round
    trip (64 encryptions, 64 plain decryptions, one launch each), RSA-2048
    CRT decryption of 16384 ciphertexts per fixed window width w = 1..6,
    exponents of 4096 / 8192 / 16128 bits on 1024 bases modulo a 2048-bit n,
    RSA-3072 / RSA-4096 CRT decryption of 4096 ciphertexts, and RSA-16384
    (encryption on the full modulus, CRT decryption, plain decryption with the
    full-length d).  HIP-event means over `--config-reps` launches after three
    untimed (one launch, after one untimed, for the plain RSA-16384
    decryption)."""
    import numpy as np
    import torch

    import gen
    from paper_1305_3699_amd import RnsContext, RsaKey

    def timed(fn, reps, warm=3):
        # untimed launches first: the first sets up the kernel's scratch and
        # the clock settles over the next few
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    reps = args.config_reps
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()
    lines = []
    # RSA-1024 round trip
    k1 = gen.rsa_key(1024, seed=gen.config_seed(1, 1))
    r1 = RsaKey(k1.n, k1.e, k1.d, k1.p, k1.q, k1.dp, k1.dq, k1.qinv)
    m1 = dev(gen.to_limbs(gen.uniform_below(k1.n, 64, seed=gen.config_seed(1, 2)), 32))
    c1 = r1.encrypt(m1)
    enc_ms = timed(lambda: r1.encrypt(m1, out=c1), reps)
    out1 = torch.empty_like(c1)
    dec_ms = timed(lambda: r1.decrypt(c1, use_crt=False, out=out1), reps)
    torch.cuda.synchronize()
    lines.append({"config": "RSA-1024, 64 messages: encrypt then plain (non-CRT) decrypt, one launch each",
                  "encrypt_ms": round(enc_ms, 4), "decrypt_ms": round(dec_ms, 4),
                  "round_trip_ok": bool(torch.equal(out1, m1))})
    # RSA-2048 CRT per window
    k2 = gen.rsa_key(2048, seed=gen.config_seed(2, 1))
    c2 = dev(gen.to_limbs(gen.uniform_below(k2.n, 16384, seed=gen.config_seed(2, 2)), 64))
    row = {"config": "RSA-2048 CRT decryption of 16384 ciphertexts, fixed window width w", "decrypts_per_s": {}}
    first = None
    agree = True
    for w in range(1, 7):
        rk = RsaKey(k2.n, k2.e, k2.d, k2.p, k2.q, k2.dp, k2.dq, k2.qinv, window=w)
        out = torch.empty_like(c2)
        ms = timed(lambda: rk.decrypt(c2, use_crt=True, out=out), reps)
        row["decrypts_per_s"][str(w)] = round(16384 / ms * 1e3, 1)
        torch.cuda.synchronize()
        if first is None:
            first = out.clone()
        agree = agree and bool(torch.equal(out, first))
        rk.close()
    row["windows_agree"] = agree   # every width's 16384 outputs bit-identical
    lines.append(row)
    # long exponents modulo a 2048-bit n
    k3 = gen.rsa_key(2048, seed=gen.config_seed(3, 1))
    ctx = RnsContext(k3.n, 64, window=6)
    x3 = dev(gen.to_limbs(gen.uniform_below(k3.n, 1024, seed=gen.config_seed(3, 2)), 64))
    row = {"config": "1024 bases modulo a 2048-bit n (k = %d), one shared exponent" % ctx.info["k"],
           "modexps_per_s": {}, "ms": {}}
    for eb in (4096, 8192, 16128):
        e = gen.random_exponent(eb, seed=gen.config_seed(3, 3) + eb)
        el = dev(gen.to_limbs(e, (eb + 31) // 32)[0])
        out = torch.empty_like(x3)
        ms = timed(lambda: ctx.modexp(x3, el, out=out), reps)
        row["modexps_per_s"][str(eb)] = round(1024 / ms * 1e3, 1)
        row["ms"][str(eb)] = round(ms, 3)
    lines.append(row)
    # RSA-3072 / RSA-4096 CRT
    row = {"config": "RSA-3072 and RSA-4096 CRT decryption of 4096 ciphertexts", "decrypts_per_s": {}, "ms": {}}
    for bits in (3072, 4096):
        k = gen.rsa_key(bits, seed=gen.config_seed(3, 10 + bits // 1024))
        rk = RsaKey(k.n, k.e, k.d, k.p, k.q, k.dp, k.dq, k.qinv)
        c = dev(gen.to_limbs(gen.uniform_below(k.n, 4096, seed=gen.config_seed(3, 20 + bits // 1024)), bits // 32))
        out = torch.empty_like(c)
        ms = timed(lambda: rk.decrypt(c, use_crt=True, out=out), reps)
        row["decrypts_per_s"][str(bits)] = round(4096 / ms * 1e3, 1)
        row["ms"][str(bits)] = round(ms, 3)
        rk.close()
    lines.append(row)
    # RSA-16384: the full modulus on 512 + 1 channels, the halves on 256 + 1
    with open(os.path.join(ROOT, "tests", "golden", "rsa16384_key.json")) as fh:
        fx = json.load(fh)
    p, q, e = int(fx["p"], 16), int(fx["q"], 16), int(fx["e"])
    n, d = p * q, pow(e, -1, (p - 1) * (q - 1))
    rk = RsaKey(n, e, d, p, q, d % (p - 1), d % (q - 1), pow(q, -1, p))
    msgs = dev(gen.to_limbs(gen.uniform_below(n, 4096, seed=gen.config_seed(8, 30)), 512))
    c = rk.encrypt(msgs)
    out = torch.empty_like(c)
    enc_ms = timed(lambda: rk.encrypt(msgs, out=out), reps)
    crt_ms = timed(lambda: rk.decrypt(c, use_crt=True, out=out), reps)
    nd = 1024
    full_ms = timed(lambda: rk.decrypt(c[:nd], use_crt=False, out=out[:nd]), 1, warm=1)
    ok = bool(torch.equal(out[:nd], msgs[:nd]))
    lines.append({"config": "RSA-16384 (stored seeded key): encryption with e = 65537 of 4096 messages on the "
                            "full modulus (k = %d), CRT decryption of the 4096 (k = %d halves), non-CRT "
                            "decryption with the full-length d of %d" % (rk.info(0)["k"], rk.info(1)["k"], nd),
                  "encrypts_per_s": round(4096 / enc_ms * 1e3, 1), "crt_decrypts_per_s": round(4096 / crt_ms * 1e3, 1),
                  "plain_decrypts_per_s": round(nd / full_ms * 1e3, 1),
                  "ms": {"encrypt": round(enc_ms, 3), "crt": round(crt_ms, 3), "plain": round(full_ms, 3)},
                  "plain_round_trip_ok": ok})
    rk.close()
    return lines


def run_tile_sweep(args) -> list:
    """Both workgroup tiles of the matrix-core kernel (16 and 32 elements) and
    the library's automatic per-launch choice, for every base size the library
    builds a kernel for, timed on batches of exponentiations by a full-length
    exponent modulo a seeded odd modulus of the size that selects that base
    (512 .. 4096 bits: the CRT halves of RSA-1024 .. RSA-8192, or the whole
    modulus of RSA-3072 / RSA-4096 with a private-size exponent), at three
    batch sizes each.  One line per (k, batch)."""
    import numpy as np
    import torch

    import gen
    from paper_1305_3699_amd import RnsContext

    lines = []
    for bits, B in ((512, 16384), (1024, 16384), (1536, 8192), (2048, 8192), (3072, 4096), (4096, 4096)):
        rng = random.Random(gen.config_seed(7, bits))
        N = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
        L = bits // 32
        e = gen.random_exponent(bits, seed=gen.config_seed(7, bits + 1))
        el = torch.from_numpy(gen.to_limbs(e, L)[0].view(np.int32)).cuda()
        x64 = torch.from_numpy(gen.to_limbs([rng.getrandbits(bits - 1) for _ in range(64)], L)
                               .view(np.int32)).cuda()
        ctxs = {g: RnsContext(N, L, group=g, window=6) for g in (16, 32, 0)}
        for batch in (B // 2, B, 2 * B):
            x = x64.repeat(batch // 64, 1).contiguous()
            out = torch.empty_like(x)
            row = {"modulus_bits": bits, "k": ctxs[0].info["k"], "batch": batch}
            for g, ctx in ctxs.items():
                ctx.modexp(x, el, out=out)
                torch.cuda.synchronize()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                for _ in range(args.tile_reps):
                    ctx.modexp(x, el, out=out)
                b.record()
                torch.cuda.synchronize()
                row["ms_%s" % (g or "auto")] = round(a.elapsed_time(b) / args.tile_reps, 3)
            print("tiles %s" % json.dumps(row), file=sys.stderr, flush=True)
            lines.append(row)
    return lines


def run_base_sweep(args) -> list:
    """The base size as a tuning dimension: batches of exponentiations by a
    full-length exponent modulo a seeded odd modulus, on the smallest base
    the modulus fits (k_min) and on each larger base the matrix engine has a
    kernel for (up to 129 channels), default tile, window 5.  The results
    must not depend on the base; one line per (modulus size, k)."""
    import numpy as np
    import torch

    import gen
    from paper_1305_3699_amd import RnsContext

    lines = []
    for bits, B in ((512, 16384), (1024, 16384), (1536, 8192), (2048, 8192)):
        rng = random.Random(gen.config_seed(8, bits))
        N = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
        L = bits // 32
        e = gen.random_exponent(bits, seed=gen.config_seed(8, bits + 1))
        el = torch.from_numpy(gen.to_limbs(e, L)[0].view(np.int32)).cuda()
        x = torch.from_numpy(gen.to_limbs([rng.getrandbits(bits - 1) for _ in range(B)], L)
                             .view(np.int32)).cuda()
        kmin = RnsContext(N, L, window=5).info["k"]
        ref = None
        for k in [k for k in (17, 33, 49, 65, 97, 129) if k >= kmin]:
            ctx = RnsContext(N, L, k=k, window=5)
            out = torch.empty_like(x)
            ctx.modexp(x, el, out=out)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(args.tile_reps):
                ctx.modexp(x, el, out=out)
            b.record()
            torch.cuda.synchronize()
            if ref is None:
                ref = out.clone()
            row = {"modulus_bits": bits, "batch": B, "k": ctx.info["k"], "k_min": kmin,
                   "group": ctx.info["group"], "ms": round(a.elapsed_time(b) / args.tile_reps, 3),
                   "same_as_k_min": bool(torch.equal(out, ref))}
            print("bases %s" % json.dumps(row), file=sys.stderr, flush=True)
            lines.append(row)
            ctx.close()
    return lines


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--window", type=int, default=5,
                    help="window width of the main workload (5: fastest in the per-width sweep of --configs)")
    ap.add_argument("--waves", type=int, default=0, help="waves per workgroup (k = 33 shapes)")
    ap.add_argument("--engine", type=int, default=0, help="0 auto, 1 channel (VALU), 2 matrix cores")
    ap.add_argument("--group", type=int, default=0, help="matrix cores: elements per workgroup (16, 32; 0 default)")
    ap.add_argument("--unscaled", action="store_true",
                    help="matrix cores: keep the key's B residues unscaled (two REDCs per quotient digit)")
    ap.add_argument("--cpu-sample", type=int, default=16384, help="ciphertexts for the oracle baseline (0: skip)")
    ap.add_argument("--sweep-window", action="store_true")
    ap.add_argument("--mixed-steps", type=int, default=5, help="timed runs of the batched-vs-plain mix (0: skip)")
    ap.add_argument("--served", action="store_true",
                    help="also run the full served sweep (5k/20k/80k req/s, 10 s each; about 2 minutes)")
    ap.add_argument("--no-served-leg", action="store_true",
                    help="skip the short served leg of the default run (80k req/s for 2 s)")
    ap.add_argument("--modmul-sweep", action="store_true",
                    help="only the 3072-bit modular multiplication sweep (one JSON line per base size)")
    ap.add_argument("--modmul-batches", type=int, nargs="+",
                    default=[16, 64, 256, 1024, 4096, 16384, 65536])
    ap.add_argument("--tile-sweep", action="store_true",
                    help="only the timing of both workgroup tiles per base size (one JSON line per k)")
    ap.add_argument("--tile-reps", type=int, default=3)
    ap.add_argument("--base-sweep", action="store_true",
                    help="time exponentiations on the smallest base a modulus fits and on each larger one")
    ap.add_argument("--configs", action="store_true",
                    help="only the other measured configurations (RSA-1024 round trip, windows, long exponents, "
                         "RSA-3072/4096 CRT)")
    ap.add_argument("--config-reps", type=int, default=5)
    ap.add_argument("--keygen", action="store_true",
                    help="only the primality steps of key generation (trial division, Miller-Rabin)")
    ap.add_argument("--keygen-candidates", type=int, default=65536)
    ap.add_argument("--keygen-mr", type=int, default=512, help="candidates given to Miller-Rabin")
    ap.add_argument("--keygen-keys", type=int, default=4, help="RSA-2048 keys generated end to end")
    ap.add_argument("--served-rates", type=float, nargs="+", default=[5000.0, 20000.0, 80000.0])
    ap.add_argument("--served-duration", type=float, default=10.0)
    ap.add_argument("--served-warmup", type=float, default=1.0)
    ap.add_argument("--served-inflight", type=int, default=4,
                    help="dispatch slots of the server (4: one per hardware queue of the process)")
    ap.add_argument("--served-max-ops", type=int, nargs="+", default=[0],
                    help="operations per dispatch at most (0: the server's default, 16384); one run per value")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one elementwise copy of N MiB before the benchmark (counter calibration)")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from rocprofv3 counter_collection.csv files")
    args = ap.parse_args(argv)
    if args.ingest_counters:
        print(json.dumps(ingest_counters(*args.ingest_counters, calib_mb=args.calib_copy_mb or 256), indent=1))
        return 0
    if args.gpus != 1:
        print("bench.py runs on one GPU only: it measures the hot path on a single device "
              "(sharding over several GPUs is described, not measured)", file=sys.stderr)
        return 2
    if args.modmul_sweep:
        for line in run_modmul_sweep(args):
            print(json.dumps(line), flush=True)
        return 0
    if args.configs:
        for line in run_configs(args):
            print(json.dumps(line), flush=True)
        return 0
    if args.keygen:
        print(json.dumps(run_keygen(args)), flush=True)
        return 0
    if args.tile_sweep:
        for line in run_tile_sweep(args):
            print(json.dumps(line), flush=True)
        return 0
    if args.base_sweep:
        for line in run_base_sweep(args):
            print(json.dumps(line), flush=True)
        return 0
    args.served_default = not args.no_served_leg and not args.sweep_window
    if args.sweep_window:
        args.mixed_steps = 0
    keys = draw_keys(args)
    if args.sweep_window:
        # the oracle runs once on the whole batch; every window's outputs are
        # compared with it
        ref = None
        for w in range(1, 7):
            args.window = w
            r, got_ref = run(argparse.Namespace(**{**vars(args), "cpu_sample": 0 if ref is not None else args.batch,
                                                   "mixed_steps": 0}), keys["c2"], ref)
            if ref is None:
                ref = got_ref
                r["matches_oracle"] = bool(r["cpu_baseline"] and r["cpu_baseline"]["matches_gpu"])
            print(json.dumps(r), flush=True)
        return 0
    out, _ = run(args, keys["c2"])
    if args.mixed_steps > 0:
        out["batched_vs_plain"] = run_mixed(args, *keys["c4"])
    if args.served_default:
        leg = argparse.Namespace(**{**vars(args), "served_rates": [80000.0], "served_duration": 2.0,
                                    "served_warmup": 0.5, "served_max_ops": [0]})
        sv = run_served(leg, keys["c5"])
        r = sv["runs"][0]
        out["served"] = {"what": "request loop over 256 resident keys (64 each of 2048/1024/3072/4096 bits), "
                                 "Poisson arrivals, 40/30/20/10%% key sizes, 70%% CRT decryptions, 64 GiB "
                                 "budget, %d slots; latency = completion - arrival (host clock), requests of "
                                 "the 0.5 s warm-up excluded" % args.served_inflight,
                         "offered_req_per_s": r["offered_req_per_s"], "duration_s": 2.0,
                         "completed_per_s": r["completed_per_s"], "latency_ms": r["latency_ms"],
                         "requests": r["requests"], "dispatches": r["dispatches"],
                         "sample_matches_oracle": r["sample_matches_oracle"]}
    if args.served:
        out["served_sweep"] = run_served(args, keys["c5"])
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
