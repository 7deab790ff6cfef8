"""Benchmark: Liouvillian applications per second on one MI355X.

Workload: the realistic synthetic cell (simple cubic a = 10.26 bohr, 48^3 grid,
ecut 25 Ha, 8 wells with s+p separable projectors, 16 bands, 8 k-points,
q = 0.2 (2 pi/a) along [100], PZ-ALDA).  One step is one full Liouvillian
application (a D step and a D+K step of the pseudo-Hermitian recursion,
every hot-path stage included), timed through lz_step with all inputs
resident on the device; the spectrum of the run is evaluated at the end.

Prints one JSON line (see the design doc for the fields).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed Liouvillian applications")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="cfg2")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "both"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stage-timing", action="store_true", default=True)
    return ap.parse_args()


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_gpu(s, prec, steps, warmup):
    import numpy as np
    import torch

    import paper_2111_06623_amd as lz
    cap = 2 * (steps + warmup) + 4
    ctx = lz.lz_init(s, prec=prec, max_steps=cap)
    ctx.step(2 * warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, st = ctx.step(2 * steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if done != 2 * (steps + warmup):
        raise RuntimeError(f"recursion stopped early at {done} steps (status {st})")
    elapsed = t1 - t0
    om = np.linspace(0.0, 2.0, 2000)
    ts = time.perf_counter()
    chi, einv, loss = ctx.spectrum(om, 0.01)
    t_spec = time.perf_counter() - ts
    # a second, shorter timed window with stage timers on
    ctx.stage_timer(True)
    ctx.step(0)
    ctx.free()
    ctx2 = lz.lz_init(s, prec=prec, max_steps=2 * 12 + 4)
    ctx2.step(2)
    ctx2.stage_timer(True)
    ctx2.step(20)
    ms, cnt = ctx2.stage_times()
    ctx2.free()
    return dict(elapsed=elapsed, applies=steps, loss=loss, chi=chi, t_spec=t_spec,
                stage_ms=ms, stage_cnt=cnt)


def stage_bytes(s, prec, ngroups):
    """Algorithmic HBM bytes of one launch of each stage (a launch covers every
    band of the instance): each array the stage must touch, read or written
    once.  c = bytes per complex, r = bytes per real; nb bands, S sticks,
    N grid points, npw the summed sphere sizes over bands and k-points."""
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
    pc = 2 * s.nks * s.nbnd * int(np.mean(s.npw_kq)) * c + 3 * npw * c
    return {
        "zfft_inv": npw * c + sticks,
        "plane_local": 2 * sticks + N * r,
        "plane_density": 2 * sticks + nb * N * c + N * r + ngroups * N * c,
        "hxc": ngroups * N * c + 7 * N * c + 2 * N * r,
        "plane_vu": nb * N * c + N * c + 2 * sticks,
        "zfft_fwd": sticks + 2 * npw * c + s.nks * int(np.mean(s.npw_kq)) * r,
        "projectors": pc,
        "lanczos": 3 * npw * c,
    }, S


def cpu_baseline(s, budget_s):
    """The oracle (unchanged) timed on the host cores: Lanczos steps on the
    same system until the time budget is spent."""
    import numpy as np  # noqa: F401
    from threadpoolctl import threadpool_limits

    import oracle.pw as opw
    from oracle import lanczos
    from oracle.liouvillian import Liouvillian
    cores = min(len(os.sched_getaffinity(0)), 16)
    opw.FFT_WORKERS = cores
    with threadpool_limits(cores):
        L = Liouvillian(s)
        y = L.rhs()
        n = 2
        t0 = time.perf_counter()
        lanczos.pseudo_hermitian_lanczos(L.apply_D, L.apply_DK, L.inner, y, n, project=L.project_c)
        dt = time.perf_counter() - t0
        while dt < budget_s / 3 and n < 64:
            n *= 2
            t0 = time.perf_counter()
            lanczos.pseudo_hermitian_lanczos(L.apply_D, L.apply_DK, L.inner, y, n, project=L.project_c)
            dt = time.perf_counter() - t0
    return dict(value=(n / 2) / dt, unit="applies/s", cores=cores, kind="oracle",
                sample=f"{n} Lanczos steps ({n // 2} applies) of the same cfg2 system, "
                       f"scipy.fft workers={cores}, BLAS threads={cores}")


def main():
    a = _args()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2111_06623_amd as lz
    from synth import config_system
    lz.load()
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible")
    t = time.perf_counter()
    s = config_system(a.config)
    _log(f"[bench] system {a.config} ready in {time.perf_counter() - t:.1f}s "
         f"(nks={s.nks}, nbnd={s.nbnd}, npw~{int(s.npw_kq.mean())}, grid={tuple(int(v) for v in s.nr)})")
    precs = ["fp64", "fp32"] if a.prec == "both" else [a.prec]
    res = {}
    for p in precs:
        _log(f"[bench] gpu {p}: warmup {a.warmup}, timed {a.steps} applies")
        res[p] = run_gpu(s, p, a.steps, a.warmup)
        _log(f"[bench] gpu {p}: {res[p]['applies'] / res[p]['elapsed']:.1f} applies/s")
    head = precs[-1]
    r = res[head]
    value = r["applies"] / r["elapsed"]
    ms_per = 1e3 * r["elapsed"] / r["applies"]
    # dominant stage and its roofline
    names = lz.STAGES
    per_launch = {names[i]: (r["stage_ms"][i] / r["stage_cnt"][i] if r["stage_cnt"][i] else 0.0)
                  for i in range(8)}
    totals = {names[i]: float(r["stage_ms"][i]) for i in range(8)}
    dom = max(totals, key=totals.get)
    ngroups = max(1, min(s.nks * s.nbnd, -(-1024 // int(s.nr[2]))))
    gsize = -(-(s.nks * s.nbnd) // ngroups)
    ngroups = -(-(s.nks * s.nbnd) // gsize)
    nbytes, nsticks = stage_bytes(s, head, ngroups)
    gbs = {k: round(nbytes[k] / (per_launch[k] * 1e-3) / 1e9, 1) for k in nbytes if per_launch.get(k, 0) > 0}
    roof = None
    if per_launch.get(dom, 0) > 0:
        ach = nbytes[dom] / (per_launch[dom] * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": 8000.0,
                "unit": "GB/s", "frac": round(ach / 8000.0, 4), "traffic": None,
                "bytes_per_launch": nbytes[dom], "avg_launch_ms": round(per_launch[dom], 5)}
    out = {
        "metric": "Liouvillian applies/s (mixed vs FP64, 1 GPU) at max spectrum rel err 1e-4",
        "value": round(value, 2), "unit": "applies/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms_per, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if head == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "cfg2: SC a=10.26 bohr, 48^3 grid, ecut 25 Ha, 8 wells + 32 s/p projectors, "
                               "16 bands, 8 k-points, q=0.2(2pi/a)[100], PZ-ALDA",
                   "precision": head, "lanczos_steps_timed": 2 * a.steps},
        "roofline": roof,
        "stage_ms_per_launch": {k: round(v, 5) for k, v in per_launch.items()},
        "stage_ms_per_apply": {k: round(totals[k] / 10.0, 5) for k in totals},
        "stage_algorithmic_GBps": gbs,
        "spectrum_ms": round(1e3 * r["t_spec"], 3),
    }
    if "fp64" in res and "fp32" in res:
        f64, f32 = res["fp64"]["loss"], res["fp32"]["loss"]
        floor = 1e-6 * np.abs(f64).max()
        out["mixed_vs_fp64"] = {
            "fp64_applies_per_s": round(res["fp64"]["applies"] / res["fp64"]["elapsed"], 2),
            "speedup": round(value / (res["fp64"]["applies"] / res["fp64"]["elapsed"]), 3),
            "loss_max_rel_err": float(np.max(np.abs(f32 - f64) / np.maximum(np.abs(f64), floor)))}
    if not a.no_cpu_baseline:
        _log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(s, a.cpu_seconds)
        out["cpu_baseline"]["value"] = round(out["cpu_baseline"]["value"], 4)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
