#!/usr/bin/env python3
"""Benchmark of the red/black Moebius CG hot path on one MI355X.

One step = one complete solve of D_DW psi = eta on the 24^3 x 64, Ls = 12
Moebius workload (b5 = 1.75, c5 = 0.75, M5 = 1.8, mf = 0.005, links
exp(i 0.6 H), Gaussian source): source preparation, CGLS on the red/black
Schur operator with an FP16-storage / FP32-arithmetic operator, FP64
reductions, reliable updates and defect correction, reconstruction and the
FP64 true-residual check (<= 1e-10).  ms_per_step is the time to solution;
value is the solve's algorithmic HBM traffic (every field read or written
once per kernel, links once per hop) divided by that time.

Also reported: the metered hop kernel (D_{p,1-p} = -1/2 H B, Sec. 3) per
precision against the 8 TB/s HBM roofline (median of 2 x 100 per-launch
event durations after 10 untimed launches), D_pre per precision, the
plain-FP64, FP32- and FP16-operator times to solution with each solution's
error against an FP64 solve to 1e-12 and the solver's condition-number
estimate, the same on 16^3 x 32, Ls = 16 with a Gaussian source, multi-RHS and
uneven-batch solves, the force, and the CPU oracle (hop, D_pre and CG on
three lattices, all threads and one) timed on the host cores.

Prints exactly one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Möbius Dslash GB/s (% HBM roofline); CG time-to-1e-10: mixed/multi-RHS vs FP64"
HBM_PEAK_GBS = 8000.0
PREC_NAMES = {0: "f64", 1: "f32", 2: "f16"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def hop_algo_bytes(op, prec):
    """In + out half spinors + one parity block of links (8 directions x Vh)."""
    from paper_1206_5214_amd import mobius
    link_elem = {mobius.F64: 16, mobius.F32: 8, mobius.F16: 4}[prec]
    return 2 * op.field_bytes(prec) + 8 * 9 * (op.V // 2) * link_elem


def time_hop(torch, op, prec, src_canon, reps=100, warm=10, opk=0):
    """Duration of each of `reps` launches per parity of the metered hop kernel
    (opk: the operator block, the hop D_{p,1-p} by default) after `warm`
    untimed ones, each bracketed by its own pair of events on the stream the
    library launches on (torch's current stream).  Returns (median, mean) in
    ms over the 2 reps launches."""
    import statistics
    even, odd = op.pack(src_canon, prec)
    out_e = op.new_field(prec)
    out_o = op.new_field(prec)
    for _ in range(warm):
        op.dslash(odd, 0, prec, out=out_e, op=opk)
        op.dslash(even, 1, prec, out=out_o, op=opk)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(2 * reps)]
    for k in range(reps):
        for j, (x, outp, out) in enumerate(((odd, 0, out_e), (even, 1, out_o))):
            a, b = ev[2 * k + j]
            a.record()
            op.dslash(x, outp, prec, out=out, op=opk)
            b.record()
    torch.cuda.synchronize()
    ms = [a.elapsed_time(b) for a, b in ev]
    del even, odd, out_e, out_o
    return statistics.median(ms), statistics.fmean(ms)


def time_schur(torch, op, prec, src_canon, reps):
    """Average duration of one D_pre application (two fused hop launches)."""
    from paper_1206_5214_amd import mobius
    _, odd = op.pack(src_canon, prec)
    out = op.new_field(prec)
    for _ in range(3):
        op.dslash(odd, 1, prec, op=mobius.OP_SCHUR, out=out)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        op.dslash(odd, 1, prec, op=mobius.OP_SCHUR, out=out)
    stop.record()
    stop.synchronize()
    ms = start.elapsed_time(stop) / reps
    del odd, out
    return ms


def copy_peak_gbs(torch, nbytes=1 << 31, reps=10):
    """Achieved rate of a plain device-to-device copy (read + write bytes)."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        b.copy_(a)
    stop.record()
    stop.synchronize()
    ms = start.elapsed_time(stop) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def counters_for(kernel_key, tuning, brick=None, auto_brick=None):
    """HBM traffic per launch measured with rocprofv3 counters, if they were
    taken on the current kernel source (profiles/<key>.json records its hash)
    with the launch parameters this run's tuner chose and the same site-order
    brick (brick None or equal to auto_brick: the automatic one)."""
    from paper_1206_5214_amd.profile_hop import hop_sources_sha256
    used = None if brick is None or list(brick) == list(auto_brick or []) else list(brick)
    # profiles/<key>.json: the automatic site order; <key>_brick<bx>x<by>x<bz>.json: another
    name = kernel_key if used is None else f"{kernel_key}_brick{'x'.join(str(b) for b in used)}"
    path = os.path.join(ROOT, "profiles", f"{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha256") != hop_sources_sha256():
        return None
    want = {k: v for k, v in tuning.items() if k != "hop_us"}
    if rec.get("tuning") is not None and rec["tuning"] != want:
        return None
    rb = rec.get("brick")
    if rb is not None and list(rb) == list(auto_brick or []):
        rb = None
    if rb != used:
        return None
    return rec.get("traffic_bytes_per_launch")


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(inputs, U2, eta2, w2):
    """The FP64 oracle, as it stands, on the host cores: one hop block and one
    D_pre application on the 4^4 (Ls 8), 16^3x32 (Ls 16) and 24^3x64 (Ls 12)
    workloads and the complete red/black CG on 4^4 with every thread; then
    one thread on the small ones (the large ones would take minutes).  A CG on
    the larger lattices takes two D_pre applications per iteration: with the
    measured D_pre and the GPU's iteration counts that is about half an hour
    (16^3x32) and hours (24^3x64) on these cores, so it is not run.  value:
    the hop on the headline lattice, GB/s by the GPU's algorithmic byte count."""
    import oracle
    nthreads = oracle.num_threads()
    out = {"nproc": os.cpu_count(), "omp_threads": nthreads, "cpu_model": _cpu_model(),
           "kind": "oracle", "runs": []}

    def hop_bytes(w):
        Vh = w.V // 2
        return 2 * Vh * w.Ls * 192 + 8 * 9 * Vh * 16

    def run(name, w, U, eta, what, threads):
        p = oracle.Params(w.dims, w.Ls, w.M5, w.mf, w.b5, w.c5)
        oracle.set_num_threads(threads)
        t0 = time.perf_counter()
        rec = {"workload": name, "what": what, "threads": threads}
        if what == "hop":
            oracle.hop(p, U, eta, 0)
            rec["GBps"] = hop_bytes(w) / (time.perf_counter() - t0) / 1e9
        elif what == "schur":
            oracle.schur(p, U, oracle.restrict(p, eta, 1))
            rec["GBps"] = (2 * hop_bytes(w) + w.V // 2 * w.Ls * 192) / (time.perf_counter() - t0) / 1e9
        else:
            _, info = oracle.solve(p, U, eta, tol=w.tol, maxiter=20000)
            rec.update(iters=info.iters, true_resid=info.true_resid)
        rec["seconds"] = time.perf_counter() - t0
        out["runs"].append(rec)
        log(f"cpu baseline: {name} {what} on {threads} threads: {rec['seconds']:.2f} s")
        return rec

    fields = {}
    for name in ("shamir_4x4x4x4_ls8", "mobius_16x16x16x32_ls16"):
        w = inputs.WORKLOADS[name]
        fields[name] = (w,) + inputs.workload_fields(w)
    fields[w2.name] = (w2, U2, eta2)
    for name in ("shamir_4x4x4x4_ls8", "mobius_16x16x16x32_ls16", w2.name):
        w, U, eta = fields[name]
        head = run(name, w, U, eta, "hop", nthreads)
        run(name, w, U, eta, "schur", nthreads)
    w, U, eta = fields["shamir_4x4x4x4_ls8"]
    run("shamir_4x4x4x4_ls8", w, U, eta, "cg", nthreads)
    for name in ("shamir_4x4x4x4_ls8", "mobius_16x16x16x32_ls16"):
        w, U, eta = fields[name]
        run(name, w, U, eta, "hop", 1)
    w, U, eta = fields["shamir_4x4x4x4_ls8"]
    run("shamir_4x4x4x4_ls8", w, U, eta, "schur", 1)
    run("shamir_4x4x4x4_ls8", w, U, eta, "cg", 1)
    oracle.set_num_threads(nthreads)
    Lx, Ly, Lz, Lt = w2.dims
    out.update(value=head["GBps"], unit="GB/s", cores=nthreads,
               sample=f"one FP64 oracle hop block D_eo on the {Lx}x{Ly}x{Lz}x{Lt}, Ls={w2.Ls} "
                      f"workload ({head['seconds']:.1f} s on {nthreads} threads); every run in 'runs'")
    return out


def point_sources_gpu(torch, dims, Ls):
    """The 12 spin-colour wall point sources at the origin, built on the device."""
    Lx, Ly, Lz, Lt = dims
    src = torch.zeros((12, Ls, Lt, Lz, Ly, Lx, 4, 3), dtype=torch.complex128, device="cuda")
    for a in range(12):
        spin, col = divmod(a, 3)
        src[a, Ls - 1 if spin < 2 else 0, 0, 0, 0, 0, spin, col] = 1.0
    return src


def _rel(torch, a, b):
    return (torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item()


def multi_rhs_runs(torch, inputs, mobius):
    """12 point sources on the multi-RHS lattice: one batched solve per inner
    precision against twelve sequential plain-FP64 solves."""
    w = inputs.MULTI_RHS
    U, _ = inputs.workload_fields(w, with_source=False)
    op = mobius.Operator(w.dims, w.Ls, w.M5, w.mf, w.b5, w.c5, torch.from_numpy(U).cuda())
    del U
    src = point_sources_gpu(torch, w.dims, w.Ls)
    out = {"workload": f"{w.name} x 12 point sources"}
    # the metered hop on this lattice too (its FP32 and FP16 working sets fit
    # the 256 MB Infinity Cache, so these rates are not HBM-bound figures)
    gauss = torch.randn(src.shape[1:], dtype=torch.complex128, device="cuda")
    hop = {}
    for prec in (mobius.F64, mobius.F32, mobius.F16):
        op.tune(prec)
        ms, _ = time_hop(torch, op, prec, gauss)
        nbytes = hop_algo_bytes(op, prec)
        hop[PREC_NAMES[prec]] = {"us": ms * 1e3, "algo_bytes": nbytes,
                                 "GBps": nbytes / (ms * 1e-3) / 1e9,
                                 "frac_hbm": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        log(f"multi-rhs lattice hop {PREC_NAMES[prec]}: {ms * 1e3:.1f} us "
            f"{hop[PREC_NAMES[prec]]['GBps']:.0f} GB/s")
    out["hop"] = hop
    del gauss
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref, iters = [], []
    for a in range(12):
        s1, i1, rc = op.solve(src[a].contiguous(), tol=w.tol, maxiter=50000, inner_prec=mobius.F64)
        if rc != mobius.OK:
            raise RuntimeError(f"FP64 solve of source {a} failed: {i1[0]}")
        ref.append(s1)
        iters.append(i1[0].iters)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    ref = torch.stack(ref)
    out["sequential_f64"] = {"seconds": seq, "iters_per_rhs": iters}
    log(f"multi-rhs: 12 sequential FP64 solves {seq:.3f} s")
    for prec, etol in ((mobius.F64, 0.0), (mobius.F32, 0.0), (mobius.F16, 0.0), (mobius.F16, 1e-8)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sol, info, rc = op.solve(src, tol=w.tol, maxiter=50000, inner_prec=prec, err_tol=etol)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if rc != mobius.OK:
            raise RuntimeError(f"batched solve failed: {info}")
        err = max(_rel(torch, sol[a], ref[a]) for a in range(12))
        name = f"batched_{PREC_NAMES[prec]}" + ("_err_tol_1e-8" if etol else "")
        out[name] = {
            "seconds": dt, "speedup_vs_sequential_f64": seq / dt,
            "max_iters": max(i.iters for i in info),
            "max_true_resid": max(i.true_resid for i in info),
            "max_rel_diff_vs_f64": err, "max_err_bound": max(i.err_bound for i in info),
            "GBps": info[0].algo_bytes / dt / 1e9}
        log(f"multi-rhs: {name} {dt:.3f} s ({seq / dt:.2f}x), "
            f"max resid {out[name]['max_true_resid']:.2e}, diff {err:.2e}")
        del sol
    # the 4d overlap propagator of the 12 spin-colour point sources at the
    # origin: D_DW(1) on the walls, one batched 5d solve, the walls read back
    Lx, Ly, Lz, Lt = w.dims
    b4 = torch.zeros((12, Lt, Lz, Ly, Lx, 4, 3), dtype=torch.complex128, device="cuda")
    for a in range(12):
        b4[a, 0, 0, 0, 0, a // 3, a % 3] = 1.0
    prop = {}
    for prec in (mobius.F64, mobius.F16):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        q, info, rc = op.propagator4d(b4, tol=w.tol, maxiter=50000, inner_prec=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if rc != mobius.OK:
            raise RuntimeError(f"4d propagator failed: {info}")
        prop[PREC_NAMES[prec]] = {"seconds": dt, "seconds_per_column": dt / 12,
                                  "max_iters": max(i.iters for i in info),
                                  "max_5d_true_resid": max(i.true_resid for i in info)}
        if prec != mobius.F64:
            prop[PREC_NAMES[prec]]["max_rel_diff_vs_f64"] = max(
                _rel(torch, q[a], q64[a]) for a in range(12))
        else:
            q64 = q
        log(f"4d propagator {PREC_NAMES[prec]}: {dt:.3f} s for 12 columns")
    out["propagator4d"] = prop
    del b4, q64
    op.close()
    return out


def uneven_batch_runs(torch, inputs, mobius):
    """8^4 + 12^4 + 16^4 (Ls = 8) in one lockstep solve against the same
    lattices solved one after another."""
    ops, srcs = [], []
    for w in inputs.UNEVEN_BATCH:
        U, eta = inputs.workload_fields(w)
        ops.append(mobius.Operator(w.dims, w.Ls, w.M5, w.mf, w.b5, w.c5, torch.from_numpy(U).cuda()))
        srcs.append(torch.from_numpy(eta).cuda())
        for prec in (mobius.F64, mobius.F32, mobius.F16):
            ops[-1].tune(prec)
    out = {"workload": " + ".join(w.name for w in inputs.UNEVEN_BATCH)}
    ref = {}
    for prec in (mobius.F64, mobius.F32):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sols = []
        for op, src in zip(ops, srcs):
            s1, i1, rc = op.solve(src, tol=1e-10, maxiter=50000, inner_prec=prec)
            if rc != mobius.OK:
                raise RuntimeError(f"solve failed: {i1[0]}")
            sols.append(s1)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ref[prec] = sols
        out[f"sequential_{PREC_NAMES[prec]}"] = {"seconds": dt}
        log(f"uneven batch: sequential {PREC_NAMES[prec]} {dt:.3f} s")
    for prec in (mobius.F64, mobius.F32, mobius.F16):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sols, infos, rc = mobius.batch_solve(ops, srcs, tol=1e-10, maxiter=50000, inner_prec=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if rc != mobius.OK:
            raise RuntimeError(f"batched solve failed: {infos}")
        err = max(_rel(torch, a, b) for a, b in zip(sols, ref[mobius.F64]))
        f64 = out["sequential_f64"]["seconds"]
        out[f"batched_{PREC_NAMES[prec]}"] = {
            "seconds": dt, "speedup_vs_sequential_f64": f64 / dt,
            "iters": [g[0].iters for g in infos],
            "max_true_resid": max(g[0].true_resid for g in infos),
            "max_rel_diff_vs_f64": err}
        log(f"uneven batch: batched {PREC_NAMES[prec]} {dt:.3f} s ({f64 / dt:.2f}x vs sequential "
            f"FP64), diff {err:.2e}")
    for op in ops:
        op.close()
    return out


def gaussian_c1_runs(torch, inputs, mobius):
    """16^3 x 32, Ls = 16, b5 = 1.5, c5 = 0.5 with a Gaussian source: plain FP64
    CG against the FP32- and FP16-operator CG with FP64 reliable updates, each
    to a 1e-10 true residual, with every solve's error against an FP64 solve
    to 1e-12."""
    w = inputs.WORKLOADS["mobius_16x16x16x32_ls16"]
    U, eta = inputs.workload_fields(w)
    op = mobius.Operator(w.dims, w.Ls, w.M5, w.mf, w.b5, w.c5, torch.from_numpy(U).cuda())
    src = torch.from_numpy(eta).cuda()
    del U, eta
    for prec in (mobius.F64, mobius.F32, mobius.F16):
        op.tune(prec)
    out = {"workload": w.name}
    ref, iref, rc = op.solve(src, tol=1e-12, maxiter=50000)
    if rc != mobius.OK:
        raise RuntimeError(f"reference solve failed: {iref}")
    for prec in (mobius.F64, mobius.F32, mobius.F16):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sol, info, rc = op.solve(src, tol=w.tol, maxiter=50000, inner_prec=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        i = info[0]
        if rc != mobius.OK:
            raise RuntimeError(f"c1 solve failed: {i}")
        out[PREC_NAMES[prec]] = {"seconds": dt, "iters": i.iters, "reliable_updates": i.reliable_updates,
                                 "true_resid": i.true_resid, "kappa": i.kappa, "err_bound": i.err_bound,
                                 "rel_error_vs_ref": _rel(torch, sol, ref)}
        log(f"c1 gaussian {PREC_NAMES[prec]}: {dt:.3f} s, {i.iters} iters, resid {i.true_resid:.2e}, "
            f"error {out[PREC_NAMES[prec]]['rel_error_vs_ref']:.2e}")
        del sol
    # the FP16 operator with the solution-error target 1e-8 as well
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol, info, rc = op.solve(src, tol=w.tol, maxiter=50000, inner_prec=mobius.F16, err_tol=1e-8)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    i = info[0]
    if rc != mobius.OK:
        raise RuntimeError(f"c1 solve with err_tol failed: {i}")
    out["f16_err_tol_1e-8"] = {"seconds": dt, "iters": i.iters, "true_resid": i.true_resid, "kappa": i.kappa,
                               "err_bound": i.err_bound, "rel_error_vs_ref": _rel(torch, sol, ref)}
    log(f"c1 gaussian f16 with err_tol 1e-8: {dt:.3f} s, {i.iters} iters, bound {i.err_bound:.2e}, "
        f"error {out['f16_err_tol_1e-8']['rel_error_vs_ref']:.2e}")
    del sol, ref
    for k in ("f32", "f16", "f16_err_tol_1e-8"):
        out[k]["speedup_vs_f64"] = out["f64"]["seconds"] / out[k]["seconds"]
    op.close()
    return out


def force_runs(torch, inputs, mobius):
    """Pseudofermion action S = phi_o^+ (D_pre^+ D_pre)^-1 phi_o with dS/dU and
    dS/dphi on the 24^3 x 64, Ls = 12 Moebius lattice (b5 = 1.5, c5 = 0.5):
    CG on the normal operator to 1e-10 (plain FP64, and FP16-storage inner
    operator with FP64 reliable updates) followed by the derivative pass."""
    w = inputs.WORKLOADS["force_24x24x24x64_ls12"]
    U, phi = inputs.workload_fields(w)
    op = mobius.Operator(w.dims, w.Ls, w.M5, w.mf, w.b5, w.c5, torch.from_numpy(U).cuda())
    phi = torch.from_numpy(phi).cuda()
    del U
    for prec in (mobius.F64, mobius.F32, mobius.F16):
        op.tune(prec)
    out = {"workload": w.name}
    ref = None
    for prec in (mobius.F64, mobius.F16):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S, G, gphi, info, rc = op.force(phi, tol=w.tol, maxiter=50000, inner_prec=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if rc != mobius.OK:
            raise RuntimeError(f"force solve failed: {info}")
        rec = {"seconds": dt, "iters": info.iters, "reliable_updates": info.reliable_updates,
               "normal_resid": info.true_resid, "action": S}
        if ref is None:
            ref = (S, G)
        else:
            rec["rel_diff_action_vs_f64"] = abs(S - ref[0]) / abs(ref[0])
            rec["max_rel_diff_grad_vs_f64"] = ((G - ref[1]).abs().max() / ref[1].abs().max()).item()
        out[f"inner_{PREC_NAMES[prec]}"] = rec
        log(f"force inner {PREC_NAMES[prec]}: {dt:.3f} s, {info.iters} iters, S = {S:.10e}")
        del G, gphi
    op.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mobius_24x24x24x64_ls12")
    ap.add_argument("--inner", default="f16", choices=["f64", "f32", "f16"])
    ap.add_argument("--hop-reps", type=int, default=100,
                    help="timed launches of the metered hop per parity (after 10 untimed)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-brick-tune", action="store_true",
                    help="keep the automatic site order instead of timing candidate bricks")
    ap.add_argument("--brick", default="",
                    help="site-order brick bx,by,bz to use without timing candidates")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the FP64 / FP32 comparison solves")
    ap.add_argument("--no-force", action="store_true",
                    help="skip the pseudofermion force timing")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the multi-RHS and uneven-batch time-to-solution runs")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(the solve of one lattice is not sharded); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1206_5214_amd import inputs, mobius

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = inputs.WORKLOADS[args.workload]
    inner = mobius.PREC[args.inner]
    log(f"workload {w.name}: dims {w.dims} Ls {w.Ls}; generating fields (seed {w.seed})")
    t0 = time.perf_counter()
    U, eta = inputs.workload_fields(w)
    log(f"fields ready in {time.perf_counter() - t0:.1f} s")
    Ud = torch.from_numpy(U).cuda()
    etad = torch.from_numpy(eta).cuda()
    # site order: the layout tuner times candidate bricks with the inner
    # operator's precision (the automatic brick unless one is > 3 % faster)
    site_order = None
    brick = None
    if args.brick:
        brick = tuple(int(b) for b in args.brick.split(","))
        site_order = {"brick": list(brick), "automatic": None, "given": True}
        log(f"site order: brick {brick} (given)")
    elif not args.no_brick_tune:
        brick, brick_us, trials = mobius.tune_brick(w.dims, w.Ls, w.M5, w.mf, w.b5, w.c5, Ud, prec=inner)
        site_order = {"brick": list(brick), "automatic": list(trials[0][0]), "hop_us": brick_us,
                      "prec": PREC_NAMES[inner],
                      "trials": [{"brick": list(b), "hop_us": u} for b, u in trials]}
        log(f"site order: brick {brick} ({brick_us:.1f} us); candidates "
            + ", ".join(f"{b}: {u:.1f}" for b, u in trials))
    op = mobius.Operator(w.dims, w.Ls, w.M5, w.mf, w.b5, w.c5, Ud, brick=brick)
    torch.cuda.synchronize()
    tuning = {}
    for prec in (mobius.F64, mobius.F32, mobius.F16):
        tuning[PREC_NAMES[prec]] = op.tune(prec)
        log(f"tuned hop {PREC_NAMES[prec]}: {tuning[PREC_NAMES[prec]]}")

    # -- metered hop kernel, every precision --------------------------------
    hop = {}
    for prec in (mobius.F64, mobius.F32, mobius.F16):
        ms, ms_mean = time_hop(torch, op, prec, etad, args.hop_reps)
        nbytes = hop_algo_bytes(op, prec)
        gbs = nbytes / (ms * 1e-3) / 1e9
        flops = 1416.0 * (op.V // 2) * w.Ls
        hop[PREC_NAMES[prec]] = {"us": ms * 1e3, "us_mean": ms_mean * 1e3, "launches": 2 * args.hop_reps,
                                 "algo_bytes": nbytes, "GBps": gbs,
                                 "frac_hbm": gbs / HBM_PEAK_GBS,
                                 "GFLOPps": flops / (ms * 1e-3) / 1e9}
        log(f"hop {PREC_NAMES[prec]}: median {ms * 1e3:.1f} us (mean {ms_mean * 1e3:.1f})  {gbs:.0f} GB/s  "
            f"({100 * gbs / HBM_PEAK_GBS:.1f}% of 8 TB/s)")
    # the hop block of the left form D^ = D-^-1 D_DW D- (Sec. 2.1), -1/2 B H:
    # the same bytes, with B applied once after the hopping sum
    hop_left = {}
    for prec in (mobius.F64, mobius.F32, mobius.F16):
        ms, ms_mean = time_hop(torch, op, prec, etad, args.hop_reps, opk=mobius.OP_HOP_LEFT)
        nbytes = hop_algo_bytes(op, prec)
        gbs = nbytes / (ms * 1e-3) / 1e9
        hop_left[PREC_NAMES[prec]] = {"us": ms * 1e3, "us_mean": ms_mean * 1e3, "launches": 2 * args.hop_reps,
                                      "algo_bytes": nbytes, "GBps": gbs, "frac_hbm": gbs / HBM_PEAK_GBS}
        log(f"left-form hop {PREC_NAMES[prec]}: median {ms * 1e3:.1f} us  {gbs:.0f} GB/s")

    # -- D_pre = 1 - I^-1 D_oe I^-1 D_eo (two fused hop launches) -----------
    schur = {}
    for prec in (mobius.F64, mobius.F32, mobius.F16):
        ms = time_schur(torch, op, prec, etad, max(10, args.hop_reps // 2))
        # in, t, t, in (subtracted), out + two link passes
        nbytes = 5 * op.field_bytes(prec) + 2 * (hop_algo_bytes(op, prec) - 2 * op.field_bytes(prec))
        gbs = nbytes / (ms * 1e-3) / 1e9
        schur[PREC_NAMES[prec]] = {"us": ms * 1e3, "algo_bytes": nbytes, "GBps": gbs,
                                   "frac_hbm": gbs / HBM_PEAK_GBS,
                                   "GFLOPps": 3048.0 * (op.V // 2) * w.Ls / (ms * 1e-3) / 1e9}
        log(f"D_pre {PREC_NAMES[prec]}: {ms * 1e3:.1f} us  {gbs:.0f} GB/s")
    copy_gbs = copy_peak_gbs(torch)
    log(f"device copy: {copy_gbs:.0f} GB/s")

    # -- the step: complete solves to 1e-10 ---------------------------------
    def solve(prec, tol=w.tol, err_tol=0.0):
        sol, info, rc = op.solve(etad, tol=tol, maxiter=50000, inner_prec=prec, err_tol=err_tol)
        i = info[0]
        if rc != mobius.OK or i.true_resid > tol:
            raise RuntimeError(f"solve did not reach {tol}: {i}")
        return sol, i

    for k in range(args.warmup):
        _, i = solve(inner)
        log(f"warmup solve {k}: {i.seconds:.3f} s, {i.iters} iters, resid {i.true_resid:.2e}")
    torch.cuda.synchronize()
    infos = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        sol, i = solve(inner)
        infos.append(i)
        log(f"timed solve {k}: {i.seconds:.3f} s, {i.iters} iters, {i.reliable_updates} reliable "
            f"updates, true resid {i.true_resid:.2e}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_per_step = 1e3 * wall / args.steps
    algo_bytes = float(np.mean([i.algo_bytes for i in infos]))
    value = algo_bytes / (ms_per_step * 1e-3) / 1e9

    compare = {}
    forms = {}
    if not args.no_compare:
        # reference: an FP64 solve to a 1e-12 true residual (its own error is
        # bounded by its kappa times that residual); every solve's error is
        # stated against it
        ref, iref = solve(mobius.F64, tol=1e-12)
        log(f"reference FP64 solve to 1e-12: {iref.iters} iters, kappa {iref.kappa:.1f}")

        def err_vs_ref(x):
            return (torch.linalg.vector_norm(x - ref) / torch.linalg.vector_norm(ref)).item()

        for prec in (mobius.F64, mobius.F32, mobius.F16):
            if prec == inner:
                s2, i2, secs = sol, infos[-1], ms_per_step * 1e-3
            else:
                s2, i2 = solve(prec)
                secs = i2.seconds
            compare[PREC_NAMES[prec]] = {"seconds": secs, "iters": i2.iters,
                                         "true_resid": i2.true_resid, "kappa": i2.kappa,
                                         "err_bound": i2.err_bound, "rel_error_vs_ref": err_vs_ref(s2)}
            log(f"compare {PREC_NAMES[prec]}: {secs:.3f} s, {i2.iters} iters, resid {i2.true_resid:.2e}, "
                f"error {compare[PREC_NAMES[prec]]['rel_error_vs_ref']:.2e} (bound {i2.err_bound:.2e})")
            if s2 is not sol:
                del s2
        f64s = compare["f64"]["seconds"]
        for k2, v in compare.items():
            v["speedup_vs_f64"] = f64s / v["seconds"]
        # the headline operator with the solution-error target 1e-8 as well
        s3, i3 = solve(inner, err_tol=1e-8)
        compare[f"{PREC_NAMES[inner]}_err_tol_1e-8"] = {
            "seconds": i3.seconds, "iters": i3.iters, "true_resid": i3.true_resid, "kappa": i3.kappa,
            "err_bound": i3.err_bound, "rel_error_vs_ref": err_vs_ref(s3),
            "speedup_vs_f64": f64s / i3.seconds}
        log(f"{PREC_NAMES[inner]} with err_tol 1e-8: {i3.seconds:.3f} s, {i3.iters} iters, bound "
            f"{i3.err_bound:.2e}, error {err_vs_ref(s3):.2e}")
        del s3
        # the same solve iterating on each form of the Schur system (Sec. 2.1, 3)
        for form, name in ((0, "left_preconditioned"), (1, "right_preconditioned"),
                           (2, "left_form_Dhat"), (3, "schur_complement")):
            s4, info4, rc4 = op.solve(etad, tol=w.tol, maxiter=50000, inner_prec=inner, form=form)
            i4 = info4[0]
            if rc4 != mobius.OK:
                raise RuntimeError(f"form {form} solve failed: {i4}")
            forms[name] = {"form": form, "seconds": i4.seconds, "iters": i4.iters, "true_resid": i4.true_resid,
                           "kappa": i4.kappa, "rel_error_vs_ref": err_vs_ref(s4)}
            log(f"form {form} ({name}): {i4.seconds:.3f} s, {i4.iters} iters, error {err_vs_ref(s4):.2e}")
            del s4
        del ref
    gaussian_c1 = None if args.no_compare else gaussian_c1_runs(torch, inputs, mobius)

    batch = None
    if not args.no_batch:
        del sol
        torch.cuda.empty_cache()
        batch = {"multi_rhs": multi_rhs_runs(torch, inputs, mobius),
                 "uneven_batch": uneven_batch_runs(torch, inputs, mobius)}
        torch.cuda.empty_cache()
    force = None
    if not args.no_force:
        force = force_runs(torch, inputs, mobius)
        torch.cuda.empty_cache()

    hname = PREC_NAMES[inner]
    key = f"hop_{hname}_{args.workload}"
    traffic = counters_for(key, tuning[hname], site_order and site_order["brick"],
                           site_order and site_order["automatic"])
    roofline = {"bound": "hbm", "achieved": hop[hname]["GBps"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": hop[hname]["GBps"] / HBM_PEAK_GBS,
                "traffic": traffic, "traffic_note": "L2-to-memory read and write requests per launch "
                "(TCC_EA0_RDREQ / WRREQ by request size) times their sizes: an upper bound on the "
                "HBM bytes (part of it is served by the Infinity Cache)",
                "kernel": f"hop_kernel {hname} (D_{{p,1-p}} = -1/2 H B)"
                          + (", colour multiply on the matrix cores" if tuning[hname].get("mfma") and
                             inner == mobius.F16 and w.Ls % 4 == 0 else ""),
                "duration": "median of per-launch HIP-event durations",
                "algo_bytes_per_launch": hop[hname]["algo_bytes"],
                "copy_GBps": copy_gbs, "frac_of_copy": hop[hname]["GBps"] / copy_gbs}

    cpu = None
    if not args.no_cpu_baseline:
        del op
        torch.cuda.empty_cache()
        cpu = cpu_baseline(inputs, U, eta, w)
        log(f"cpu baseline: {cpu['value']:.3f} GB/s on {cpu['cores']} threads ({cpu['sample']})")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if inner != mobius.F64 else "f64",
        "storage": hname,
        "data": "synthetic (seeded exp(i eps H) SU(3) links, Gaussian source)",
        "config": {"workload": w.name, "dims": list(w.dims), "Ls": w.Ls, "M5": w.M5, "mf": w.mf,
                   "b5": w.b5, "c5": w.c5, "link_eps": w.eps, "seed": w.seed, "tol": w.tol,
                   "inner_prec": hname, "reductions": "f64"},
        "solve": {"iters": infos[-1].iters, "reliable_updates": infos[-1].reliable_updates,
                  "true_resid": infos[-1].true_resid, "kappa": infos[-1].kappa,
                  "err_bound": infos[-1].err_bound, "algo_bytes": algo_bytes,
                  "GFLOPps": float(np.mean([i.flops for i in infos])) / (ms_per_step * 1e-3) / 1e9},
        "dslash": {"kernel": f"hop {hname}", "GBps": hop[hname]["GBps"],
                   "frac_hbm": hop[hname]["frac_hbm"], "GFLOPps": hop[hname]["GFLOPps"]},
        "hop": hop,
        "hop_left_form": hop_left,
        "schur": schur,
        "solve_forms": forms,
        "time_to_solution": compare,
        "gaussian_16x16x16x32_ls16": gaussian_c1,
        "batched": batch,
        "force": force,
        "tuning": tuning,
        "site_order": site_order,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
