"""Benchmark: Liouvillian applications per second on one MI355X.

Workload: the realistic synthetic cell (simple cubic a = 10.26 bohr, 48^3 grid,
ecut 25 Ha, 8 Gaussian wells with 32 s+p separable projectors, 16 bands,
8 k-points, q = 0.2 (2 pi/a) along [100], Perdew-Zunger ALDA), recursions of
1000 Lanczos steps; the mixed-precision variant of the same cell is defined at
3000 steps.

One step of the metric is one full Liouvillian application: a D step and a
D+K step of the pseudo-Hermitian recursion, with every hot-path stage (sticks
and plane FFTs, local potential, projectors, response density, Hartree + xc,
P_c, Lanczos scalars).  Each precision is timed over 5 windows of complete
recursions (each restarted from (0, y) and followed by its spectrum on 2000
frequencies; a window holds at least 1000 Lanczos steps and at least --steps
applications), inputs resident on the device; the median window is reported.

The headline is the fastest path whose loss function meets the metric's gate:
within 1e-4 of the FP64 oracle (relative, floored at 1e-6 of the maximum) at
the recursion length of its configuration -- 3000 steps for the mixed path,
1000 for the FP64 path.  The oracle's loss at 300, 1000 and 3000 steps is read
from tests/golden/cfg2_oracle_reference.npz.  Every path's error at every
length is reported, with the error that a 1e-12 relative perturbation of the
local potential alone causes in the FP64 path (without reorthogonalisation
the recursion amplifies any perturbation once Ritz values converge).

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

OMEGA = (0.0, 2.0, 2000)
ETA = 0.01
GATE = 1e-4
WINDOWS = 5
RAW_APPLIES = 200   # raw lz_apply_liouvillian calls timed per precision
REFERENCE = os.path.join(ROOT, "tests", "golden", "cfg2_oracle_reference.npz")
# recursion length of each precision's configuration (the gate is taken there)
CONFIG_STEPS = {"fp64": 1000, "fp32": 3000, "splitbf16": 3000}
GATE_LENGTHS = (300, 1000, 3000)


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=150,
                    help="Liouvillian applications per timed window at least (a window also holds "
                         "at least one complete recursion)")
    ap.add_argument("--warmup", type=int, default=10, help="untimed Liouvillian applications")
    ap.add_argument("--config", default="cfg2")
    ap.add_argument("--prec", default="all", choices=["fp64", "fp32", "splitbf16", "all"])
    ap.add_argument("--lanczos-steps", type=int, default=1000,
                    help="steps of one timed recursion (the workload's 1000)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="budget of the oracle samples")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gates", action="store_true",
                    help="skip the 3000-step error runs (timing only)")
    ap.add_argument("--apply-stages", default=None, metavar="CONFIG",
                    help="only time the stages of operator applications on CONFIG (e.g. cfg5r)")
    ap.add_argument("--batched", type=int, default=0, metavar="N",
                    help="only time the first N members of the batched uneven workload")
    ap.add_argument("--ground-state", default=None, metavar="CONFIG",
                    help="only time the device ground-state preparation on CONFIG")
    ap.add_argument("--large-cell", type=int, default=0, metavar="STEPS",
                    help="only the large cell (96^3, 128 bands, 4 k) from device-prepared orbitals: "
                         "recursions of STEPS steps in FP64, FP32 and split bf16")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this size (counter calibration)")
    ap.add_argument("--nh-steps", type=int, default=60,
                    help="steps of the per-step comparison with the non-Hermitian recursion (0: skip)")
    ap.add_argument("--sweep-steps", type=int, default=200,
                    help="steps of the q-sweep throughput comparison (0: skip)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="the built-in launch heuristics instead of the autotuner at init")
    ap.add_argument("--graph", action="store_true",
                    help="replay pairs of steps as captured graphs (measured no faster than eager)")
    return ap.parse_args()


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_jobs(ctx, nsteps, M, om):
    """nsteps Lanczos steps as complete recursions of M steps (the last one
    shorter if M does not divide nsteps), each followed by its spectrum."""
    left = nsteps
    while left > 0:
        n = min(M, left)
        ctx.reset()
        done, _ = ctx.step(n)
        if done != n:
            raise RuntimeError(f"recursion stopped at {done} of {n} steps")
        ctx.spectrum(om, ETA, m=n)
        left -= n


# stages that are a single kernel launch each (the roofline is quoted on one)
SINGLE_KERNEL = ("zfft_inv", "plane_local", "plane_density", "plane_vu", "zfft_fwd")


def loss_err(loss, ref):
    """max over omega of |loss - ref| / max(|ref|, 1e-6 max|ref|)."""
    import numpy as np
    floor = 1e-6 * np.abs(ref).max()
    return float(np.max(np.abs(loss - ref) / np.maximum(np.abs(ref), floor)))


def run_gpu(s, prec, applies, warmup, M, graph, autotune=True):
    """Median of WINDOWS timed windows of complete M-step recursions (each
    window at least `applies` applications), after warm-up and autotuning;
    per-stage times from a short window with every stage timed; the dominant
    single-kernel stage timed with HIP events inside the timed windows."""
    import numpy as np
    import torch

    import paper_2111_06623_amd as lz
    om = np.linspace(*OMEGA)
    ctx = lz.lz_init(s, prec=prec, max_steps=max(M, 32) + 2, use_graph=graph, autotune=autotune)
    run_jobs(ctx, 2 * warmup, M, om)
    ctx.reset()
    ctx.step(2)
    ctx.stage_timer(True)
    ctx.step(20)
    ms, cnt = ctx.stage_times()
    dom = max(SINGLE_KERNEL, key=lambda n: ms[lz.STAGES.index(n)])
    per_window = max(2 * applies, M)
    windows = []
    ctx.stage_timer(True, stages=[dom])
    for _ in range(WINDOWS):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_jobs(ctx, per_window, M, om)
        torch.cuda.synchronize()
        windows.append(time.perf_counter() - t0)
    dms, dcnt = ctx.stage_times()
    ctx.stage_timer(False)
    di = lz.STAGES.index(dom)
    # raw operator applications (lz_apply_liouvillian, a D and a D+K half on
    # device vectors), outside the recursion
    x = torch.randn(sum(ctx.nvec), dtype=torch.complex128 if prec == "fp64" else torch.complex64,
                    device="cuda")
    qo, po = torch.empty_like(x), torch.empty_like(x)
    for _ in range(5):
        ctx.apply_liouvillian(x, x, qo, po)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for _ in range(RAW_APPLIES):
        ctx.apply_liouvillian(x, x, qo, po)
    torch.cuda.synchronize()
    raw_rate = RAW_APPLIES / (time.perf_counter() - ta)
    del x, qo, po
    ctx.reset()
    ctx.step(M)
    ts = time.perf_counter()
    ctx.spectrum(om, ETA, m=M)
    t_spec = time.perf_counter() - ts
    tuning = ctx.tuning()
    ctx.free()
    med = float(np.median(windows))
    return dict(window_s=windows, median_s=med, applies=per_window // 2,
                rate=(per_window / 2) / med, t_spec=t_spec, stage_ms=ms, tuning=tuning,
                stage_cnt=cnt, dom=dom, dom_ms=dms[di] / max(dcnt[di], 1),
                dom_launches=int(dcnt[di]), raw_rate=raw_rate)


def error_profile(s, prec, ref, lengths, perturb=0.0):
    """Loss functions of one recursion of max(lengths) steps at every length,
    their errors against the oracle's stored loss (ref: the reference file)
    or, with ref None, the raw losses; beta over the first 50 steps; the
    largest |Im z| / max|z|.  perturb scales the local potential by
    (1 + perturb) (a probe of how the recursion amplifies a perturbation)."""
    import copy

    import numpy as np

    import paper_2111_06623_amd as lz
    if perturb:
        s = copy.copy(s)
        s.vloc_r = np.asarray(s.vloc_r) * (1.0 + perturb)
    om = np.linspace(*OMEGA)
    mmax = max(lengths)
    ctx = lz.lz_init(s, prec=prec, max_steps=mmax + 2)
    done = 0
    out = {"loss": {}}
    for m in sorted(lengths):
        d, _ = ctx.step(m - done)
        if d != m:
            raise RuntimeError(f"{prec} recursion stopped at {d} of {m} steps")
        done = m
        out["loss"][m] = ctx.spectrum(om, ETA, m=m)[2]
    beta, _, z = ctx.coefficients()
    ctx.free()
    out["beta"] = beta
    out["im_z_rel"] = float(np.abs(z.imag).max() / np.abs(z).max())
    if ref is not None:
        out["loss_err"] = {m: loss_err(out["loss"][m], ref[f"loss_{m}"]) for m in lengths}
        nb = 50
        out["beta50_err"] = float(np.max(np.abs(beta[:nb] - ref["beta"][:nb]) / ref["beta"][:nb]))
    return out


def load_reference(s):
    """The oracle's stored recursion of the 48^3 cell, if it belongs to s."""
    import numpy as np
    if not os.path.exists(REFERENCE):
        return None
    r = np.load(REFERENCE, allow_pickle=False)
    same = (np.array_equal(r["npw_kq"], s.npw_kq) and r["et_k"].shape == s.et_k.shape
            and np.abs(r["et_k"] - s.et_k).max() < 1e-10)
    return {k: r[k] for k in r.files} if same else None


def nh_vs_ph(s, prec, steps):
    """Wall time per Lanczos step of the pseudo-Hermitian and the non-Hermitian
    recursions on the same system and precision (steps after a few warmup
    steps, device synchronised on both sides; outside the timed region of the
    headline metric)."""
    import torch

    import paper_2111_06623_amd as lz
    out = {"precision": prec, "steps": steps}
    for alg in ("ph", "nh"):
        ctx = lz.lz_init(s, prec=prec, max_steps=steps + 8, algorithm=alg)
        ctx.step(4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done, _ = ctx.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if done != steps + 4:
            raise RuntimeError(f"{alg} recursion stopped at {done} steps")
        out[f"{alg}_ms_per_step"] = round(1e3 * dt / steps, 4)
        ctx.free()
    out["nh_over_ph"] = round(out["nh_ms_per_step"] / out["ph_ms_per_step"], 3)
    return out


def q_sweep_rate(systems, prec, steps):
    """Instance-applies/s of a q-dispersion sweep (the 32^3 crystal at eight
    q along [100], one instance per q, in one context): the instances one
    after another on one stream against side by side on the library's
    default streams, each with and without graph replay, and one launch per
    kernel of a step over all eight (batched).  Outside the timed region of
    the headline metric."""
    import torch

    import paper_2111_06623_amd as lz
    out = {"workload": "q sweep: 32^3 cell (cfg2 crystal at ecut 8 Ha, 16 bands, 2 k) at "
                       "q = (0.05..0.6) 2pi/a [100], 8 instances", "precision": prec,
           "instances": len(systems), "steps": steps}
    modes = [(1, False, False, "one_stream"), (1, True, False, "one_stream_graph"),
             (0, False, False, "side_by_side"), (0, True, False, "side_by_side_graph"),
             (1, False, True, "one_launch"), (1, True, True, "one_launch_graph")]
    for streams, graph, batched, key in modes:
        ctx = lz.lz_init(systems, prec=prec, max_steps=steps + 8, use_graph=graph,
                         streams=streams, batched=batched)
        ctx.step(4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done, _ = ctx.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if done != steps + 4:
            raise RuntimeError(f"sweep stopped at {done} steps")
        out[key] = round(len(systems) * steps / 2 / dt, 1)
        ctx.free()
    out["unit"] = "instance-applies/s"
    return out


def apply_stages(config, precs, reps=5):
    """Per-stage cost of lz_apply_liouvillian (both halves: a D and a D+K
    application) on one workload, for the large cells that do not run the
    recursion here (cfg5r has random orbitals).  Stage times come from HIP
    events on the library's stream; the projector products are also given
    in TFLOP/s against the precision's dense matrix-core peak."""
    import numpy as np
    import torch

    import paper_2111_06623_amd as lz
    from synth import config_system
    s = config_system(config)
    peak = {"fp64": 78.6, "fp32": 157.3, "splitbf16": 2500.0 / 3.0}
    out = {"workload": config, "nr": [int(v) for v in s.nr], "nks": int(s.nks),
           "nbnd": int(s.nbnd), "nproj": int(s.nproj), "npwx": int(s.nl_kq.shape[1])}
    npw = int(np.sum(s.npw_kq))
    # complex multiply-adds of the four projector products of both halves:
    # per half the input dot (nbnd + nproj rows), input P_c update (nbnd),
    # output dot (nbnd) and output update (nbnd + nproj), each 8 flops
    ptot = s.nbnd + s.nproj
    flops = 2 * 8.0 * npw * s.nbnd * (ptot + s.nbnd + s.nbnd + ptot)
    for prec in precs:
        ctx = lz.lz_init(s, prec=prec, max_steps=4)
        dt = torch.complex128 if prec == "fp64" else torch.complex64
        x = torch.randn(sum(ctx.nvec), dtype=dt, device="cuda")
        qo, po = torch.empty_like(x), torch.empty_like(x)
        for _ in range(2):
            ctx.apply_liouvillian(x, x, qo, po)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.apply_liouvillian(x, x, qo, po)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        ctx.stage_timer(True)
        for _ in range(reps):
            ctx.apply_liouvillian(x, x, qo, po)
        torch.cuda.synchronize()
        ms, cnt = ctx.stage_times()
        ctx.stage_timer(False)
        st = {n: round(float(m) / reps, 4) for n, m in zip(lz.STAGES, ms) if cnt[lz.STAGES.index(n)]}
        pr = st.get("projectors", 0.0)
        out[prec] = {"ms_per_apply": round(1e3 * wall, 3), "stage_ms_per_apply": st,
                     "projector_tflops": round(flops / (pr * 1e-3) / 1e12, 1) if pr else None,
                     "projector_frac_of_matrix_peak":
                         round(flops / (pr * 1e-3) / 1e12 / peak[prec], 3) if pr else None}
        _log(f"[bench] {config} {prec}: {out[prec]}")
        ctx.free()
    print(json.dumps(out), flush=True)


def ground_state_time(config):
    """Wall time of the device ground-state preparation on the k+q spheres
    of a workload (LOBPCG to residual 1e-9), with its eigenvalue error
    against the dense diagonalisation that built the synthetic system."""
    import numpy as np
    import torch

    import paper_2111_06623_amd as lz
    from synth import config_system
    s = config_system(config)
    nb = s.evc_kq.shape[1]
    lz.lz_ground_state(s, n_extra=4, tol=1e-6, max_iter=3)  # warm-up (kernel loading)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evc, eps, it, res = lz.lz_ground_state(s, n_extra=4, tol=1e-9)
    dt = time.perf_counter() - t0
    out = {"workload": config, "nks": int(s.nks), "nbnd": int(nb), "npwx": int(s.nl_kq.shape[1]),
           "iterations": it, "max_residual": res, "seconds": round(dt, 4),
           "max_eig_err_Ha": float(np.abs(eps - s.et_kq[:, :nb]).max())}
    print(json.dumps(out), flush=True)


def batched_rate(n_inst, prec="fp32", reps=5, steps=100):
    """Instance-applies/s of the batched uneven workload: the first n_inst
    seeded members (grids in {32, 40, 48, 64, 72}, 8-48 bands, 1-16 k-points;
    seeded orthonormal orbitals with energies below a lower bound of H, so
    that D is positive definite) in one context: recursions of `steps` steps
    of every member (lz_step), and operator applications
    (lz_apply_liouvillian), one instance after another on one stream against
    side by side on the library's streams; the recursions also with one
    launch per kernel of a step over every member of a group of instances
    that issue the same kernels (batched), the groups one after another or
    side by side."""
    import torch

    import paper_2111_06623_amd as lz
    from synth import config_system
    t = time.perf_counter()
    systems = []
    for i in range(n_inst):
        systems.append(config_system("uneven", index=i))
        if i % 8 == 7:
            _log(f"[bench] {i + 1} batched members built in {time.perf_counter() - t:.1f}s")
    out = {"workload": f"batched uneven: members 0..{n_inst - 1}", "instances": n_inst,
           "precision": prec, "steps": steps, "reps": reps,
           "grids": [int(s.nr[0]) for s in systems],
           "band_k_products": [int(s.nks) * int(s.evc_kq.shape[1]) for s in systems]}
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    modes = [(1, False, "one_stream"), (0, False, "side_by_side"), (1, True, "one_launch"),
             (0, True, "one_launch_side_by_side")]
    for streams, batched, tag in modes:
        ctx = lz.lz_init(systems, prec=prec, max_steps=steps + 4, streams=streams, batched=batched)
        ctx.step(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            ctx.step(steps)
        except lz.LzError as e:  # an instance whose metric is indefinite stops; the rest go on
            _log(f"[bench] {tag}: {e}")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        done = [ctx.state(i) for i in range(n_inst)]
        out[f"recursion_{tag}"] = round(sum(min(d, steps + 2) - 2 for d, _ in done) / 2 / el, 2)
        out[f"recursion_{tag}_stopped"] = [i for i, (d, st) in enumerate(done) if st != 0]
        if batched:  # operator applications are not batched: the per-instance figures hold
            ctx.free()
            continue
        x = torch.randn(sum(ctx.nvec), dtype=dt, device="cuda")
        qo, po = torch.empty_like(x), torch.empty_like(x)
        ctx.apply_liouvillian(x, x, qo, po)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.apply_liouvillian(x, x, qo, po)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[f"apply_{tag}"] = round(n_inst * reps / el, 2)
        ctx.free()
        del x, qo, po
    out["unit"] = "instance-applies/s"
    print(json.dumps(out), flush=True)


def large_cell(steps):
    """The large cell end to end: the lowest 128 eigenpairs of its k and k+q
    spheres, the density and f_xc on the device, then one recursion of
    `steps` steps per precision with its spectrum.  Reported: the ground-state
    time, applies/s per precision, per-stage times and their fraction of the
    HBM peak on the stick-model bytes, and the loss error of the mixed paths
    against the FP64 path (the oracle's own run of this length is out of
    reach on the host; its first 50 steps pin the FP64 path, tests)."""
    import copy

    import numpy as np
    import torch

    from synth import config_system, k_sphere_system
    s = config_system("cfg5r")
    sk = k_sphere_system("cfg5r")
    import paper_2111_06623_amd as lz
    lz.load()
    out = {"workload": "cfg5: SC a=20.5 bohr, 96^3 grid, ecut 25 Ha, 64 wells + 256 s/p projectors, "
                       "128 bands, 4 k-points, q=(0.2,0.1,0)(2pi/a), PZ-ALDA; orbitals, density and "
                       "f_xc prepared on the device", "steps": steps}
    t0 = time.perf_counter()
    evc_kq, eps_kq, it1, res1 = lz.lz_ground_state(s, n_extra=4, tol=1e-9)
    evc_k, eps_k, it2, res2 = lz.lz_ground_state(sk, n_extra=4, tol=1e-9)
    g = copy.copy(s)
    g.evc_k, g.evc_kq, g.et_k = evc_k, evc_kq, eps_k
    n0, fxc = lz.lz_ground_density(g, xc="pz")
    g.fxc_r = fxc
    torch.cuda.synchronize()
    out["ground_state"] = {"seconds": round(time.perf_counter() - t0, 2), "iterations": [it1, it2],
                           "max_residual": max(res1, res2)}
    _log(f"[bench] large cell: ground state in {out['ground_state']['seconds']} s "
         f"({it1}, {it2} iterations)")
    om = np.linspace(*OMEGA)
    losses = {}
    for prec in ("fp64", "fp32", "splitbf16"):
        ctx = lz.lz_init(g, prec=prec, max_steps=steps + 24)
        ctx.step(2)
        ctx.stage_timer(True)
        ctx.step(20)
        ms, cnt = ctx.stage_times()
        ctx.stage_timer(False)
        ctx.reset()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        done, _ = ctx.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        if done != steps:
            raise RuntimeError(f"{prec} recursion stopped at {done} of {steps} steps")
        losses[prec] = ctx.spectrum(om, ETA, m=steps)[2]
        gsize = ctx.tuning()[1]
        ctx.free()
        ngroups = -(-(s.nks * s.nbnd) // gsize)
        model, impl, _ = stage_bytes(s, prec, ngroups)
        per_launch = {lz.STAGES[i]: (ms[i] / cnt[i] if cnt[i] else 0.0) for i in range(8)}
        out[prec] = {"applies_per_s": round((steps / 2) / dt, 3), "ms_per_apply": round(2e3 * dt / steps, 3),
                     "stage_ms_per_launch": {k: round(v, 4) for k, v in per_launch.items()},
                     "stage_frac_of_hbm_peak_model_bytes":
                         {k: round(model[k] / (per_launch[k] * 1e-3) / 8e12, 4)
                          for k in model if per_launch.get(k, 0) > 0 and k != "lanczos"}}
        if prec != "fp64":
            out[prec]["loss_err_vs_fp64_gpu"] = loss_err(losses[prec], losses["fp64"])
        _log(f"[bench] large cell {prec}: {out[prec]['applies_per_s']} applies/s")
    print(json.dumps(out), flush=True)


def kernel_sources_sha():
    """sha256 over the kernel sources; a change invalidates counter data."""
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2111_06623_amd", "csrc")
    for f in sorted(os.listdir(src)):
        with open(os.path.join(src, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(stage, config, prec):
    """HBM bytes per launch from the committed counter summary of this kernel
    and workload, or None if there is none or the kernels changed since."""
    import re
    path = os.path.join(ROOT, "profiles", f"traffic_{stage}_{config}_{prec}.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_sha = re.search(r"kernel_sources_sha256\s*\|\s*([0-9a-f]{64})", txt)
    m_b = re.search(r"hbm_bytes_per_launch\s*\|\s*([0-9.eE+]+)", txt)
    if not m_sha or not m_b or m_sha.group(1) != kernel_sources_sha():
        return None
    return float(m_b.group(1))


def copy_probe(mib, launches):
    """A plain device copy of known size (calibration of the HBM counters)."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(launches):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_per_launch": 4 * n, "launches": launches}), flush=True)


def stage_bytes(s, prec, ngroups):
    """HBM bytes of one launch of each stage (a launch covers every band of
    the instance), two ways.  c = bytes per complex, r = bytes per real; nb
    bands, S sticks, N3 points per stick, N grid points, npw the summed
    sphere sizes over bands and k-points.

    model: the algorithmic count of a stick-pruned two-pass transform
    with the valence orbitals held as z-transformed sticks: every stick
    volume (nb N3 S c) moved once per pass -- D: inverse z 1, plane pass 2,
    forward z 1; D+K: inverse z 1, density pass 3 (x, u, V x), v'u pass 3
    (u, V x, out), forward z 1 -- plus the sphere I/O, V_loc, one n' and one
    v' grid, f_xc and the Hartree kernel.

    impl: what these kernels read and write by design: the valence orbitals
    as real-space grids (nb N c) in the density and v'u passes, the band-group
    partial densities (G N c) of the fixed-order reduction, and the Hartree
    line passes' intermediate grids."""
    import numpy as np
    c = 16 if prec == "fp64" else 8
    r = c // 2
    nb = s.nks * s.nbnd
    n1, n2, n3 = (int(v) for v in s.nr)
    cols = set()
    for k in range(s.nks):
        for nl, npw in ((s.nl_k[k], s.npw_k[k]), (s.nl_kq[k], s.npw_kq[k])):
            cols.update((np.asarray(nl[:npw]) // n3).tolist())
    S = len(cols)
    npw = int(np.sum(s.npw_kq)) * s.nbnd
    N = n1 * n2 * n3
    sticks = nb * n3 * S * c
    ptot = s.nbnd + s.nproj
    kin = s.nks * int(np.mean(s.npw_kq)) * r
    proj = s.nks * ptot * int(np.mean(s.npw_kq)) * c * 2 + 3 * npw * c
    model = {
        "zfft_inv": npw * c + sticks,
        "plane_local": 2 * sticks + N * r,
        "plane_density": 3 * sticks + N * r + N * c,
        "hxc": 2 * N * c + 2 * N * r,
        "plane_vu": 3 * sticks + N * c,
        "zfft_fwd": sticks + 2 * npw * c + kin,
        "projectors": proj,
        "lanczos": 3 * npw * c,
    }
    impl = dict(model)
    impl["plane_density"] = 2 * sticks + nb * N * c + N * r + ngroups * N * c
    impl["hxc"] = ngroups * N * c + 7 * N * c + 2 * N * r
    impl["plane_vu"] = nb * N * c + N * c + 2 * sticks
    return model, impl, S


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(s, budget_s):
    """The oracle (unchanged) timed on the host cores, single-threaded and on
    all cores (at most 16, the CPU share of one GPU): Lanczos steps on the
    same system, doubling the count until a third of each half of the budget
    is spent.  Building the oracle's operator (valence orbitals in real
    space) is outside the timing."""
    from threadpoolctl import threadpool_limits

    import oracle.pw as opw
    from oracle import lanczos
    from oracle.liouvillian import Liouvillian
    cores = min(len(os.sched_getaffinity(0)), 16)
    out = {}
    for tag, th in (("single", 1), ("all", cores)):
        opw.FFT_WORKERS = th
        with threadpool_limits(th):
            L = Liouvillian(s)
            y = L.rhs()
            n = 2
            t0 = time.perf_counter()
            lanczos.pseudo_hermitian_lanczos(L.apply_D, L.apply_DK, L.inner, y, n, project=L.project_c)
            dt = time.perf_counter() - t0
            while dt < budget_s / 6 and n < 64:
                n *= 2
                t0 = time.perf_counter()
                lanczos.pseudo_hermitian_lanczos(L.apply_D, L.apply_DK, L.inner, y, n,
                                                 project=L.project_c)
                dt = time.perf_counter() - t0
        out[tag] = dict(value=round((n / 2) / dt, 4), threads=th, steps=n)
    opw.FFT_WORKERS = 1
    a = out["all"]
    return dict(value=a["value"], unit="applies/s", cores=cores, kind="oracle",
                sample=f"{a['steps']} Lanczos steps ({a['steps'] // 2} applies) of the same system, "
                       f"scipy.fft workers={cores}, BLAS threads={cores}; single thread: "
                       f"{out['single']['steps']} steps",
                single_thread=dict(value=out["single"]["value"], unit="applies/s", cores=1),
                cpu_model=_cpu_model())


def main():
    a = _args()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}), flush=True)
        sys.exit(2)
    if a.copy_probe_mib:
        copy_probe(a.copy_probe_mib, 8)
        return
    if a.batched:
        import paper_2111_06623_amd as lz
        lz.load()
        batched_rate(a.batched, "fp64" if a.prec == "fp64" else "fp32")
        return
    if a.ground_state:
        import paper_2111_06623_amd as lz
        lz.load()
        ground_state_time(a.ground_state)
        return
    if a.large_cell:
        large_cell(a.large_cell)
        return
    if a.apply_stages:
        import paper_2111_06623_amd as lz
        lz.load()
        precs = ["fp64", "fp32", "splitbf16"] if a.prec == "all" else [a.prec]
        apply_stages(a.apply_stages, precs)
        return
    import numpy as np

    from synth import config_system, q_sweep
    # every synthetic system is built before the first GPU call (the input
    # preparation uses worker processes)
    t = time.perf_counter()
    s = config_system(a.config)
    sweep_systems = q_sweep("cfg2lo") if a.sweep_steps > 0 else None
    ref = load_reference(s) if a.config == "cfg2" else None
    _log(f"[bench] system {a.config} ready in {time.perf_counter() - t:.1f}s "
         f"(nks={s.nks}, nbnd={s.nbnd}, npw~{int(s.npw_kq.mean())}, grid={tuple(int(v) for v in s.nr)}); "
         f"oracle reference {'loaded' if ref is not None else 'absent'}")
    import torch

    import paper_2111_06623_amd as lz
    lz.load()
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible")
    precs = ["fp64", "fp32", "splitbf16"] if a.prec == "all" else [a.prec]
    M = a.lanczos_steps
    res = {}
    for p in precs:
        _log(f"[bench] gpu {p}: warmup {a.warmup} applies, {WINDOWS} windows of "
             f">= {max(a.steps, M // 2)} applies, recursions of {M} steps")
        res[p] = run_gpu(s, p, a.steps, a.warmup, M, a.graph, not a.no_autotune)
        _log(f"[bench] gpu {p}: {res[p]['rate']:.1f} applies/s (windows "
             f"{', '.join(f'{w * 1e3:.1f}' for w in res[p]['window_s'])} ms)")
    # errors against the oracle at every length, and the amplification probe
    errors, gates = {}, {}
    if not a.no_gates:
        for p in precs:
            _log(f"[bench] error profile {p}: {max(GATE_LENGTHS)} steps")
            errors[p] = error_profile(s, p, ref, GATE_LENGTHS)
        if "fp64" in precs:
            _log("[bench] error profile fp64 with V_loc (1 + 1e-12)")
            pert = error_profile(s, "fp64", None, GATE_LENGTHS, perturb=1e-12)
            base = errors["fp64"]["loss"]
            errors["fp64_perturbed"] = {m: loss_err(pert["loss"][m], base[m]) for m in GATE_LENGTHS}
        for p in precs:
            e = errors[p].get("loss_err")
            if e is None:  # no stored oracle: the FP64 path is the labelled stand-in
                if p == "fp64":
                    gates[p] = {"reference": "none stored (the FP64 path is the reference)",
                                "pass": True, "im_z_over_max_z": errors[p]["im_z_rel"]}
                    continue
                if "fp64" not in errors:
                    continue
                e = {m: loss_err(errors[p]["loss"][m], errors["fp64"]["loss"][m]) for m in GATE_LENGTHS}
            m = CONFIG_STEPS[p]
            gates[p] = {"reference": "oracle" if ref is not None else "fp64 gpu path",
                        "steps": m, "max_rel_err": e[m], "threshold": GATE, "pass": e[m] <= GATE,
                        "err_by_steps": {str(k): v for k, v in e.items()},
                        "beta50_rel_err": errors[p].get("beta50_err"),
                        "im_z_over_max_z": errors[p]["im_z_rel"]}
    passing = [p for p in precs if gates.get(p, {}).get("pass", not gates)]
    head = max(passing, key=lambda p: res[p]["rate"]) if passing else "fp64" if "fp64" in res else precs[0]
    r = res[head]
    value = r["rate"]
    names = lz.STAGES
    per_launch = {names[i]: (r["stage_ms"][i] / r["stage_cnt"][i] if r["stage_cnt"][i] else 0.0)
                  for i in range(8)}
    dom = r["dom"]
    gsize = r["tuning"][1]  # bands per density group, as the library chose
    ngroups = -(-(s.nks * s.nbnd) // gsize)
    model, impl, nstick = stage_bytes(s, head, ngroups)
    # (the Lanczos stage times the scalar finalisation only: its vector
    # updates are fused into the projector passes, so it has no byte model)
    frac_model = {k: round(model[k] / (per_launch[k] * 1e-3) / 8e12, 4)
                  for k in model if per_launch.get(k, 0) > 0 and k != "lanczos"}
    roof = None
    if r["dom_ms"] > 0:
        ach = model[dom] / (r["dom_ms"] * 1e-3) / 1e9
        traffic = measured_traffic(dom, a.config, head)
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": 8000.0,
                "unit": "GB/s", "frac": round(ach / 8000.0, 4), "traffic": traffic,
                "bytes_per_launch": model[dom], "bytes_model": "orbitals as z-transformed sticks",
                "impl_bytes_per_launch": impl[dom],
                "impl_over_model": round(impl[dom] / model[dom], 3),
                "traffic_over_model": round(traffic / model[dom], 3) if traffic else None,
                "avg_launch_ms": round(r["dom_ms"], 5), "timed_launches": r["dom_launches"]}
    wl = ("cfg2: SC a=10.26 bohr, 48^3 grid, ecut 25 Ha, 8 wells + 32 s/p projectors, 16 bands, "
          "8 k-points, q=0.2(2pi/a)[100], PZ-ALDA" if a.config == "cfg2" else a.config)
    out = {
        "metric": "Liouvillian applies/s (mixed vs FP64, 1 GPU) at max spectrum rel err 1e-4",
        "value": round(value, 2), "unit": "applies/s", "n_gpus": 1, "steps": r["applies"],
        "warmup": a.warmup, "ms_per_step": round(1e3 / value, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if head == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": wl, "precision": head, "lanczos_steps_per_recursion": M,
                   "timing": f"median of {WINDOWS} windows of {r['applies']} applies",
                   "graph": a.graph, "autotune": not a.no_autotune,
                   "tuning": {p: dict(zip(("projector_gemm", "density_group_bands", "projector_chunks", "fft_planes"),
                                          res[p]["tuning"])) for p in res},
                   "spectrum": "2000 frequencies in [0, 2] Ha, eta 0.01 Ha"},
        "roofline": roof,
        "rates": {p: {"applies_per_s": round(res[p]["rate"], 2),
                      "window_ms": [round(w * 1e3, 2) for w in res[p]["window_s"]],
                      "raw_apply_liouvillian_per_s": round(res[p]["raw_rate"], 2)} for p in res},
        "gates": gates,
        "stage_ms_per_launch": {k: round(v, 5) for k, v in per_launch.items()},
        "stage_frac_of_hbm_peak_model_bytes": frac_model,
        "sticks": nstick,
        "spectrum_ms": round(1e3 * r["t_spec"], 3),
    }
    if "fp64_perturbed" in errors:
        out["fp64_amplification"] = {
            "what": "loss error of the FP64 path with V_loc scaled by (1 + 1e-12) against the "
                    "unperturbed FP64 path, by recursion length",
            "err_by_steps": {str(k): v for k, v in errors["fp64_perturbed"].items()}}
    if "fp64" in res and len(res) > 1:
        out["mixed_vs_fp64"] = {p: round(res[p]["rate"] / res["fp64"]["rate"], 3)
                                for p in res if p != "fp64"}
    if a.nh_steps > 0:
        _log(f"[bench] per-step cost: pseudo-Hermitian vs non-Hermitian, {a.nh_steps} steps ({head})")
        out["nh_vs_ph"] = nh_vs_ph(s, head, a.nh_steps)
        _log(f"[bench] {out['nh_vs_ph']}")
    if sweep_systems:
        _log(f"[bench] q sweep, {a.sweep_steps} steps (fp32)")
        out["q_sweep"] = q_sweep_rate(sweep_systems, "fp32", a.sweep_steps)
        _log(f"[bench] {out['q_sweep']}")
    if not a.no_cpu_baseline:
        _log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(s, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
