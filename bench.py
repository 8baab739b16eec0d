#!/usr/bin/env python3
"""Throughput of trajectory-unravelled tVMC on one MI355X.

A step is one Heun step of every trajectory of the workload: noise, then for the predictor and
the corrector Metropolis sampling, local estimators, D, S + eps I, the FP64 Cholesky solve and
the update; moments of the collective spin are recorded every `obs_every` steps from the
predictor samples and the learned proposal is retrained every `ar_train_every` steps, as in a
production run.  value = trajectory-steps per second with every input already resident in HBM.
The default workload is the N = 64 open chain with the RBM ansatz (M = 4224), 8192 samples and
64 trajectories, learned proposal, BF16-split matrix-core S and FP64 solve; `plain_form_value`
is the same workload in the plain form (FP64 S, single-flip proposal, one trajectory per
launch).

Extra objects on the JSON line:
  roofline      the dominant kernel's algorithmic work per launch over its average launch time
                (HIP events on the library's stream inside the timed region) against the peak
                of the unit it runs on;
  cpu_baseline  the FP64 oracle on a bounded sample of the same workload, on the host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# CPU threads the oracle baseline may use: one GPU's share of the host (the GPU hosts allot 16
# CPUs per GPU, whatever the machine's total count is)
CPU_SHARE = 16

PEAKS = {  # MI355X published dense peaks
    "fp64": 78.6,            # TFLOP/s, vector and matrix
    "int8": 5000.0,          # TOP/s, matrix cores
    "bf16": 2500.0,          # TFLOP/s, matrix cores
    "hbm": 8000.0,           # GB/s
}


def kernel_sources_sha() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2506_23928_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str):
    """HBM bytes per launch from profiles/hbm_traffic_<kernel>.txt, if it was measured on the
    current kernel sources (key=value lines written from rocprofv3 --pmc runs)."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_%s.txt" % kernel)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha") != kernel_sources_sha():
        return None
    try:
        return float(kv["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def ansatz_of(tv, w):
    """(kind, n_hidden, M, theta0) of a workload."""
    import workloads as wl
    if w.get("ansatz", "jastrow") == "rbm":
        nh = w["n_hidden"]
        return tv.RBM, nh, tv.n_params(tv.RBM, w["n"], nh), wl.rbm_theta0(w["n"], nh, w["w_scale"], w["seed"])
    if w.get("ansatz") == "ljph":
        return tv.LJPH, w["d"], tv.n_params(tv.LJPH, w["n"], w["d"]), None
    return tv.JASTROW, 0, tv.n_params(tv.JASTROW, w["n"]), None


def build_context(tv, w, precision, n_traj=None, traj_offset=0, proposal=None, solver=0, regulariser=0, graph=False,
                  sampler_chains=0):
    from paper_2506_23928_amd.problem import kac_couplings
    import workloads as wl
    lx, ly = wl.lattice(w)
    J = kac_couplings(w["geom"], lx, w["alpha"], w["jscale"], ly)
    prob = tv.Problem(J, w["h"], wl.jumps(w))
    steps = wl.n_steps(w)
    kind, nh, _, th0 = ansatz_of(tv, w)
    if proposal is None:
        proposal = tv.PROPOSAL_LEARNED if w.get("proposal") == "learned" else tv.PROPOSAL_FLIP
    cfg = tv.make_config(n_traj or w["n_traj"], w["n_samples"], w["n_chains"], w["dt"], w["diag_shift"],
                         w["burn_sweeps"], w["thin_sweeps"], 0, tv.HEUN, precision, w["obs_every"],
                         steps // w["obs_every"] + 2, w["seed"], traj_offset, proposal=proposal,
                         ar_hidden=w.get("ar_hidden", 128), ar_train_every=w.get("ar_train_every", 20),
                         ar_train_iters=w.get("ar_train_iters", 50), ar_lr=w.get("ar_lr", 3e-3), solver=solver,
                         regulariser=regulariser, snr_tau=w.get("snr_tau", 4.0), use_graph=graph,
                         sampler_chains=sampler_chains)
    return tv.Context(prob, cfg, kind=kind, n_hidden=nh, theta0=th0)


def cpu_baseline(w, ns_sample=None, regulariser=0):
    """The oracle as it stands on a bounded sample: P host threads, each running one predictor
    evaluation of its own trajectory (sampling, local estimators, S, F, N^n, D, Cholesky solve);
    one trajectory-step is two evaluations.  With ns_sample below the workload's sample count
    the oracle's own phase timers scale the sample-linear phases (sampling and estimators;
    means, S, F, N^n, D) by n_samples / ns_sample, and the solve is taken as measured."""
    import numpy as np
    import oracle as orc
    import workloads as wl
    cores = min(len(os.sched_getaffinity(0)), CPU_SHARE)
    lx, ly = wl.lattice(w)
    J = orc.couplings(w["geom"], lx, w["alpha"], w["jscale"], ly)
    pb = orc.Problem(J, w["h"], wl.jumps(w))
    rbm = w.get("ansatz", "jastrow") == "rbm"
    kind, nh = (1, w["n_hidden"]) if rbm else (2, w["d"]) if w.get("ansatz") == "ljph" else (0, 0)
    m = orc.n_params(kind, w["n"], nh)
    th0 = wl.rbm_theta0(w["n"], nh, w["w_scale"], w["seed"]) if rbm else np.zeros(m)
    ns_full = w["n_samples"]
    ns = ns_sample or ns_full
    cfg = orc.Config(n_samples=ns, n_chains=w["n_chains"], burn_sweeps=w["burn_sweeps"],
                     thin_sweeps=w["thin_sweeps"], dt=w["dt"], diag_shift=w["diag_shift"], seed=w["seed"],
                     regulariser=regulariser, snr_tau=w.get("snr_tau", 4.0))
    times = []

    def work(traj):
        ch = orc.init_chains(w["seed"], traj, w["n"], w["n_chains"])
        dw = orc.draw_dw(w["seed"], traj, 0, len(wl.jumps(w)), w["dt"])
        r = orc.evaluate(pb, kind, nh, cfg, th0, ch, traj=traj, first=True, dw=dw, want_moments=False)
        sec = r["seconds"]
        times.append((sec[0] + sec[1]) * ns_full / ns + sec[2])

    t0 = time.perf_counter()
    ths = [threading.Thread(target=work, args=(t,)) for t in range(cores)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    el = time.perf_counter() - t0
    t_eval = sum(times) / len(times)
    if ns == ns_full:
        sample = ("%d trajectories x 1 predictor evaluation (half a Heun step) of %s, one per host thread, "
                  "%.1f s wall" % (cores, w["name"], el))
    else:
        sample = ("%d trajectories x 1 predictor evaluation of %s with %d of its %d samples, one per host thread "
                  "(%.1f s wall); sampling, estimators, S, F, N^n and D scaled by %d (linear in the samples), "
                  "the Cholesky solve as measured: %.1f s per full evaluation" % (
                      cores, w["name"], ns, ns_full, el, ns_full // ns, t_eval))
    return {"value": cores / t_eval / 2.0, "unit": "trajectory-steps/s", "cores": cores, "kind": "oracle",
            "sample": sample, "host_cpus": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0)),
            "cpu_model": cpu_model(), "per_core": 1.0 / t_eval / 2.0}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# kernels that time as one group (a secondary entry skips the dominant one's group)
_KERNELS_OF = {"solve": ("k_zmw_solve", "k_cmw_solve", "k_chol_solve", "k_jacobi"),
               "sbuild": ("k_sbuild_rbm_bf16", "k_sbuild_rbm_f64", "k_sbuild_f64", "k_sbuild_i8", "k_tk_rbm"),
               "transpose": ("k_rbm_split",)}


def roofline_of(tv, groups, kind, prec, ss, m, ns, nh, T, reg, solver_arg, group=None, n=64):
    """A kernel group's algorithmic work per launch (every trajectory of the context) over its
    average launch time (HIP events on the library's stream), against the peak of the unit it
    runs on: the dominant group (largest total time), or `group`."""
    dom = group or (max(groups, key=lambda g: groups[g]["total_ms"]) if groups else None)   # None: untimed
    dim = ns if ss else m                 # dimension of the system solved
    if dom == "solve" and reg == tv.tvmc.REG_SNR:
        # Jacobi: per sweep M' - 1 rounds rotating every row of S and V^T and every column of S
        # (12 flops per rotated pair of entries); the sweep count is not known here, so the
        # figure is per sweep and the fraction is left out
        roof = {"kernel": "k_jacobi", "bound": "alu", "achieved": None, "peak": PEAKS["fp64"], "unit": "TFLOP/s",
                "frac": None, "traffic": None, "note": "SNR solve: Jacobi sweeps until converged"}
    elif dom == "solve":
        if kind == tv.RBM:   # complex Hermitian Cholesky (4/3 n^3 real flops) and two triangular solves
            flops = T * (4.0 * dim ** 3 / 3.0 + 16.0 * dim * dim)
            kname = "k_zmw_solve"     # k_zmw_init, k_zmw_update(_lds), k_zmw_diag, k_zmw_bwd
        else:
            flops = T * (dim ** 3 / 3.0 + dim * dim / 2.0 + dim / 6.0 + 4.0 * dim * dim)
            multi = solver_arg == "multi" or (solver_arg != "one" and T < 192)
            kname = "k_cmw_solve" if multi else "k_chol_solve"   # k_cmw_*: the several-workgroup launches
        if ss:               # push-back delta = A^H u: M x N_s complex multiply-adds
            flops += T * 8.0 * m * ns
        achieved = flops / (groups["solve"]["avg_ms"] * 1e-3) / 1e12
        roof = {"kernel": kname, "bound": "mfma", "achieved": achieved, "peak": PEAKS["fp64"],
                "unit": "TFLOP/s", "frac": achieved / PEAKS["fp64"], "traffic": read_traffic(kname),
                "note": "one evaluation's solve (every launch of the solver for all trajectories)"}
    elif dom == "sbuild" and ss and kind == tv.RBM:
        # K = (1 + q)(1 + g) - 1 with g = t t^H over N' hidden units, Hermitian: N_s (N_s + 1) / 2
        # entries of N' complex multiply-adds (FP64 matrix cores); the group also holds the
        # centring passes over K (row means, T = H K H / N_s + eps I)
        flops = T * 8.0 * ns * (ns + 1) / 2.0 * nh
        achieved = flops / (groups["sbuild"]["avg_ms"] * 1e-3) / 1e12
        roof = {"kernel": "k_tk_rbm", "bound": "mfma", "achieved": achieved, "peak": PEAKS["fp64"],
                "unit": "TFLOP/s", "frac": achieved / PEAKS["fp64"], "traffic": read_traffic("k_tk_rbm"),
                "note": "the K-build group: the Gram on the matrix cores and the centring passes"}
    elif dom == "sbuild" and kind == tv.RBM and prec == tv.PREC_MFMA:
        # complex Hermitian S: M (M + 1) / 2 entries, N_s complex multiply-adds (8 flops) each,
        # on BF16 matrix cores (three split products per real product)
        flops = T * (m * (m + 1) / 2.0) * ns * 8.0
        achieved = flops / (groups["sbuild"]["avg_ms"] * 1e-3) / 1e12
        roof = {"kernel": "k_sbuild_rbm_bf16", "bound": "mfma", "achieved": achieved, "peak": PEAKS["bf16"] / 3.0,
                "unit": "TFLOP/s", "frac": achieved / (PEAKS["bf16"] / 3.0), "traffic": read_traffic("k_sbuild_rbm_bf16"),
                "note": "peak = BF16 dense peak / 3 (three split products per real product)"}
    elif dom == "sbuild" and kind == tv.RBM:
        # complex Hermitian S: M (M + 1) / 2 entries, N_s complex multiply-adds (8 flops) each
        flops = T * (m * (m + 1) / 2.0) * ns * 8.0
        achieved = flops / (groups["sbuild"]["avg_ms"] * 1e-3) / 1e12
        roof = {"kernel": "k_sbuild_rbm_f64", "bound": "alu", "achieved": achieved, "peak": PEAKS["fp64"],
                "unit": "TFLOP/s", "frac": achieved / PEAKS["fp64"], "traffic": read_traffic("k_sbuild_rbm_f64")}
    elif dom == "sbuild" and not ss and prec == tv.PREC_FP64:
        flops = T * (m * (m + 1) / 2.0) * ns * 2.0
        achieved = flops / (groups["sbuild"]["avg_ms"] * 1e-3) / 1e12
        roof = {"kernel": "k_sbuild_f64", "bound": "alu", "achieved": achieved, "peak": PEAKS["fp64"],
                "unit": "TFLOP/s", "frac": achieved / PEAKS["fp64"], "traffic": read_traffic("k_sbuild_f64")}
    elif dom == "sbuild" and not ss:
        ops = T * (m * (m + 1) / 2.0) * ns * 2.0
        achieved = ops / (groups["sbuild"]["avg_ms"] * 1e-3) / 1e12
        roof = {"kernel": "k_sbuild_i8", "bound": "mfma", "achieved": achieved, "peak": PEAKS["int8"],
                "unit": "TOP/s", "frac": achieved / PEAKS["int8"], "traffic": read_traffic("k_sbuild_i8")}
    elif dom == "transpose" and kind == tv.RBM and prec == tv.PREC_MFMA and not ss:
        # k_rbm_split: reads the samples (ceil(N/64) words each), tanh(theta_h) (N' complex per
        # sample) and <O> (M complex), writes the four BF16 planes of Mp x N_s
        words, mp = (n + 63) // 64, (m + 127) // 128 * 128
        nbytes = T * (ns * words * 8.0 + ns * nh * 16.0 + m * 16.0 + mp * ns * 8.0)
        achieved = nbytes / (groups["transpose"]["avg_ms"] * 1e-3) / 1e9
        roof = {"kernel": "k_rbm_split", "bound": "hbm", "achieved": achieved, "peak": PEAKS["hbm"], "unit": "GB/s",
                "frac": achieved / PEAKS["hbm"], "traffic": read_traffic("k_rbm_split")}
    else:
        roof = {"kernel": dom, "bound": "alu", "achieved": None, "peak": None, "unit": None, "frac": None,
                "traffic": None}
    return roof


def tau_int(series):
    """Integrated autocorrelation time of chains' time series [C][L] (mean over chains of the
    normalised autocorrelation, summed with Sokal's self-consistent window W >= 5 tau)."""
    import numpy as np
    x = np.asarray(series, dtype=np.float64)
    x = x - x.mean(axis=1, keepdims=True)
    var = (x * x).mean()
    if var == 0.0:
        return 0.5
    L = x.shape[1]
    tau = 0.5
    for k in range(1, L // 2):
        tau += (x[:, :-k] * x[:, k:]).mean() / var
        if k >= 5 * tau:
            break
    return tau


def autocorrelation(tv, w, steps, n_traj):
    """tau_int of Re E_loc and of M_z along each Markov chain, learned proposal against single
    flips, after `steps` SDE steps (the network retrained every ar_train_every steps)."""
    import numpy as np
    from paper_2506_23928_amd import tvmc as T
    out = {}
    for label, prop in (("learned", tv.PROPOSAL_LEARNED), ("flip", tv.PROPOSAL_FLIP)):
        ctx = build_context(tv, w, tv.PREC_MFMA, n_traj=n_traj, proposal=prop)
        ctx.sde_step(steps)
        ctx.sample()
        ctx.synchronize()
        nc, per, n = w["n_chains"], w["n_samples"] // w["n_chains"], w["n"]
        te, tm = [], []
        for t in range(n_traj):
            e = ctx.get(T.Q_ELOC, t).real.reshape(nc, per)
            s = tv.unpack_samples(ctx.get(T.Q_SAMPLES, t), n).astype(np.float64).sum(axis=1).reshape(nc, per)
            te.append(tau_int(e))
            tm.append(tau_int(s))
        out[label] = {"tau_eloc": float(np.mean(te)), "tau_mz": float(np.mean(tm)),
                      "accept_learned": (float(np.mean([ctx.get(T.Q_AR_ACCEPTS, t).mean() for t in range(n_traj)]))
                                         if prop == tv.PROPOSAL_LEARNED else None)}
        del ctx
    return out


APPD_REFERENCE = {"chain64_rbm_learned": "chain64_obc_a1.5_g0.1"}


def load_appd(workload):
    """App. D's exact xi^2 at the output times (tests/golden/appd_<case>.txt, written from the
    oracle by tests/golden/make_appd_reference.py): {t: xi^2}."""
    path = os.path.join(ROOT, "tests", "golden", "appd_%s.txt" % APPD_REFERENCE[workload])
    out = {}
    for line in open(path):
        if line.startswith("#"):
            continue
        v = [float(x) for x in line.split()]
        out[round(v[0], 6)] = v[-1]
    return out


def jackknife_sigma(loo):
    import numpy as np
    loo = np.asarray(loo, dtype=np.float64)
    T = loo.shape[0]
    return float(np.sqrt((T - 1) / T * np.sum((loo - loo.mean(axis=0)) ** 2, axis=0)))


# forms of the error protocol: (S-build precision, proposal)
FORMS = {"plain": ("fp64", "flip"), "precision": ("mfma", "flip"), "fast": ("mfma", "learned")}


def error_run(tv, w, form, ns, out_dir, dt=None, max_seconds=None, resume_dir=None):
    """One form of the fixed-xi^2-error protocol: every trajectory of the workload from t = 0 to
    t_end with N_s samples per evaluation, moments every obs_every steps; xi^2 at each output
    time from the library's trajectory average, with a jackknife over the trajectories (each
    leave-one-out ensemble on the GPU), and e = max_t |xi^2(t) - xi^2_exact(t)| with its own
    jackknife sigma.  Writes <out_dir>/error_<form>_<ns>[_dt<dt>].json.  With max_seconds, a run
    that has not finished after that much wall time stops at the next output time and leaves a
    checkpoint (tvmc_save_state) and its elapsed time in out_dir; the same call resumes from it
    (found in out_dir or resume_dir)."""
    import numpy as np
    import workloads as wl
    prec, prop = FORMS[form]
    ww = dict(w)
    ww["n_samples"] = ns
    if dt:
        ww["dt"] = dt
        ww["obs_every"] = int(round(0.1 / dt))
    tag = "%s_%d" % (form, ns) + ("_dt%g" % dt if dt else "")
    exact = load_appd(w["name"])
    ctx = build_context(tv, ww, tv.PREC_MFMA if prec == "mfma" else tv.PREC_FP64,
                        proposal=tv.PROPOSAL_LEARNED if prop == "learned" else tv.PROPOSAL_FLIP)
    steps, every, T = wl.n_steps(ww), ww["obs_every"], ww["n_traj"]
    os.makedirs(out_dir, exist_ok=True)
    ckpt, part = os.path.join(out_dir, "ckpt_%s.npy" % tag), os.path.join(out_dir, "partial_%s.json" % tag)
    el0, start = 0.0, 0
    if resume_dir and not os.path.exists(ckpt):
        ckpt_in, part_in = (os.path.join(resume_dir, os.path.basename(x)) for x in (ckpt, part))
    else:
        ckpt_in, part_in = ckpt, part
    if os.path.exists(ckpt_in) and os.path.exists(part_in):
        ctx.load_state(np.load(ckpt_in))
        start = ctx.position()[0]
        el0 = json.load(open(part_in))["seconds"]
        print("error protocol: %s resumed at step %d" % (tag, start), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for s0 in range(start, steps, every):
        ctx.sde_step(every)
        ctx.synchronize()
        print("error protocol: %s step %d of %d (%.0f s)" % (tag, s0 + every, steps, time.perf_counter() - t0),
              file=sys.stderr, flush=True)
        if max_seconds and s0 + every < steps and time.perf_counter() - t0 > max_seconds:
            np.save(ckpt, ctx.save_state())
            with open(part, "w") as f:
                json.dump({"seconds": el0 + time.perf_counter() - t0, "step": s0 + every}, f)
            print(json.dumps({"form": form, "n_samples": ns, "checkpoint_step": s0 + every}), flush=True)
            return None
    el = el0 + time.perf_counter() - t0
    ctx.sample()
    ctx.observables()
    ctx.synchronize()
    times, xi, sig, dev, loo_dev, mx = [], [], [], [], [], []
    for k in range(1, steps // every + 1):
        slot = k if k < steps // every else -1          # record k holds step k * every; the last is the final pass
        t = round(k * every * ww["dt"], 6)
        M, C, x2, loo = ctx.ensemble_at(slot, jackknife=True)
        times.append(t)
        xi.append(x2)
        mx.append(float(M[0]))
        sig.append(jackknife_sigma(loo))
        dev.append(x2 - exact[t])
        loo_dev.append(loo - exact[t])
    loo_dev = np.abs(np.array(loo_dev))                  # [times][T]
    e = float(np.max(np.abs(dev)))
    res = {"workload": w["name"], "form": form, "s_build": prec, "proposal": prop, "n_samples": ns, "n_traj": T,
           "steps": steps, "dt": ww["dt"], "seconds": el, "traj_steps_per_s": T * steps / el, "t": times,
           "xi2": xi, "xi2_sigma": sig, "xi2_exact": [exact[t] for t in times], "mx": mx, "e": e,
           "e_sigma": jackknife_sigma(loo_dev.max(axis=0)), "t_of_e": times[int(np.argmax(np.abs(dev)))],
           "kernel_sources_sha": kernel_sources_sha()}
    with open(os.path.join(out_dir, "error_%s.json" % tag), "w") as f:
        json.dump(res, f)
    for fn in (ckpt, part):
        if os.path.exists(fn):
            os.remove(fn)
    print(json.dumps({k: res[k] for k in ("form", "n_samples", "e", "e_sigma", "t_of_e", "traj_steps_per_s")}),
          flush=True)
    del ctx
    return res


def error_summary(in_dir, workload, autocorr_path=None):
    """The fixed-xi^2-error protocol from the --error-run results in in_dir: the plain form (FP64
    S, single flips) at the workload's N_s gives e_plain; the fast form (BF16-split S, learned
    proposal) is taken at the smallest N_s whose e_fast <= e_plain + 2 sigma_e, sigma_e the
    jackknife errors of the two e added in quadrature.  Returns the summary dict."""
    import glob
    runs = [json.load(open(f)) for f in sorted(glob.glob(os.path.join(in_dir, "error_*.json")))]
    runs = [r for r in runs if r["workload"] == workload]
    import workloads as wl
    ns0, dt0 = wl.WORKLOADS[workload]["n_samples"], wl.WORKLOADS[workload]["dt"]
    plain = [r for r in runs if r["form"] == "plain" and r["n_samples"] == ns0 and r["dt"] == dt0][0]
    fast = sorted([r for r in runs if r["form"] == "fast" and r["dt"] == dt0], key=lambda r: r["n_samples"])
    rows = []
    for r in runs:
        rows.append({k: r[k] for k in ("form", "n_samples", "dt", "e", "e_sigma", "t_of_e", "traj_steps_per_s", "t",
                                       "xi2", "xi2_sigma", "xi2_exact", "mx", "kernel_sources_sha")})
    ok = []
    for r in fast:
        sig = (plain["e_sigma"] ** 2 + r["e_sigma"] ** 2) ** 0.5
        r["equal_error"] = r["e"] <= plain["e"] + 2.0 * sig
        r["sigma_e"] = sig
        if r["equal_error"]:
            ok.append(r)
    star = ok[0] if ok else None
    out = {"workload": workload, "protocol": "e = max over t in 0.1..t_end of |xi^2 - xi^2_exact(App. D)|, jackknife "
           "over trajectories; fast form accepted when e_fast <= e_plain + 2 sigma_e",
           "n_samples_plain": plain["n_samples"], "e_plain": plain["e"], "e_plain_sigma": plain["e_sigma"],
           "fast": [{"n_samples": r["n_samples"], "e": r["e"], "e_sigma": r["e_sigma"], "sigma_e": r["sigma_e"],
                     "equal_error": r["equal_error"], "traj_steps_per_s": r["traj_steps_per_s"]} for r in fast],
           "n_samples_fast": star["n_samples"] if star else None, "e_fast": star["e"] if star else None,
           "runs": rows}
    if autocorr_path and os.path.exists(autocorr_path):
        out["autocorr"] = json.load(open(autocorr_path))
    return out


def bench_uneven(tv, args):
    """The uneven batch: 512 trajectories of open chains with N drawn from {16, 24, 32, 48, 64},
    alpha and gamma per trajectory (all-pair Jastrow, 2048 samples, int8 S-build), one context per
    N on its own stream, optionally with each group's plain steps replayed from a captured HIP
    graph and each group's forms and sampler workgroup shape from the autotuner's cache.  Timed:
    K whole steps of every trajectory; then two eager steps with per-kernel HIP events give the
    kernel times of every group and the roofline of the busiest group's dominant kernel."""
    import torch
    import workloads as wl
    from paper_2506_23928_amd.problem import litf_problem
    from paper_2506_23928_amd.uneven import UnevenBatch
    w = wl.UNEVEN
    params = wl.uneven_params(w["n_traj"], seed=w["seed"])
    probs = [litf_problem(n, a, w["h"], g) for n, a, g in params]
    conf = dict(n_samples=w["n_samples"], n_chains=w["n_chains"], dt=w["dt"], diag_shift=w["diag_shift"],
                seed=w["seed"], precision=tv.PREC_MFMA, burn_sweeps=w["burn_sweeps"], thin_sweeps=w["thin_sweeps"],
                use_graph=int(args.graph))
    print("bench: uneven batch of %d trajectories, N in %s, graph=%d, autotune=%s" % (
        w["n_traj"], w["sizes"], int(args.graph), args.autotune), file=sys.stderr, flush=True)
    ub = UnevenBatch(probs, autotune=args.autotune, **conf)
    ub.sde_step(max(args.warmup, 1))
    ub.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ub.sde_step(args.steps)
    ub.synchronize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    value = w["n_traj"] * args.steps / el
    print("bench: %d steps in %.3f s -> %.1f trajectory-steps/s" % (args.steps, el, value), file=sys.stderr,
          flush=True)
    per_n, busiest = {}, None
    for n, members, ctx in ub.groups:
        ctx.set_timing(True)
    ub.sde_step(2)
    ub.synchronize()
    for n, members, ctx in ub.groups:
        gms = {}
        for g in ("sample", "estimate", "transpose", "sbuild", "solve", "update"):
            ms, cnt = ctx.timing(g)
            if cnt:
                gms[g] = {"avg_ms": ms, "launches": cnt, "total_ms": ms * cnt}
        ctx.set_timing(False)
        tot = sum(v["total_ms"] for v in gms.values())
        per_n[n] = {"n_traj": len(members), "n_params": ctx.m, "sample_space": bool(ctx.sample_space),
                    "choice": {k: int(getattr(ctx.config, k)) for k in ("solver", "precision", "sampler_chains")},
                    "kernel_ms": {g: round(v["avg_ms"], 4) for g, v in gms.items()}, "ms_per_step": tot / 2}
        if busiest is None or tot > busiest[0]:
            busiest = (tot, n, ctx, gms)
    _, n, ctx, gms = busiest
    roof = roofline_of(tv, gms, tv.JASTROW, tv.PREC_MFMA, ctx.sample_space, ctx.m, w["n_samples"], 0,
                       ctx.config.n_traj, tv.tvmc.REG_SHIFT, "auto")
    roof["group"] = "N = %d" % n
    out = {"metric": "trajectory-steps/s, uneven batch (512 trajectories, N in {16, 24, 32, 48, 64})", "value": value,
           "unit": "trajectory-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": el / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "uneven", "n_traj": w["n_traj"], "sizes": list(w["sizes"]), "n_samples": w["n_samples"],
                      "n_chains": w["n_chains"], "dt": w["dt"], "ansatz": "jastrow", "s_build": "int8 MFMA (exact)",
                      "graph": bool(args.graph), "autotune": bool(args.autotune)},
           "roofline": roof, "groups": {str(k): v for k, v in per_n.items()},
           "kernel_sources_sha": kernel_sources_sha()}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="chain64_rbm_learned")
    ap.add_argument("--precision", choices=["mfma", "fp64"], default="mfma")
    ap.add_argument("--sampler-chains", type=int, default=0,
                    help="Markov chains per sampler workgroup (1, 2, 4, 8, 16; 0: the library's choice)")
    ap.add_argument("--solver", choices=["auto", "one", "multi"], default="auto",
                    help="FP64 Cholesky with one or several workgroups per trajectory (auto: by batch size)")
    ap.add_argument("--regulariser", choices=["shift", "snr"], default="shift",
                    help="diagonal shift (Cholesky) or the SNR filter in S's eigenbasis (Jastrow ansaetze)")
    ap.add_argument("--autotune", metavar="JSON", default=None,
                    help="--workload uneven: take each group's forms and sampler shape from this autotuner cache "
                         "(tuned and written there first when missing)")
    ap.add_argument("--graph", action="store_true",
                    help="replay one captured HIP graph per plain step (per-kernel timing is then off)")
    ap.add_argument("--log", metavar="FILE",
                    help="run --steps steps, appending per-step metrics as JSON lines to FILE (untimed)")
    ap.add_argument("--autocorr", action="store_true",
                    help="measure the integrated autocorrelation time with and without the learned proposal")
    ap.add_argument("--error-run", metavar="FORM:NS",
                    help="one form of the fixed-xi^2-error protocol (plain, precision or fast, at NS samples, "
                         "optionally FORM:NS:DT): the "
                         "whole run against App. D, written as JSON to --out")
    ap.add_argument("--out", default="gpurun_out", help="directory of --error-run results")
    ap.add_argument("--max-seconds", type=float, default=None,
                    help="--error-run: checkpoint and stop after this much wall time (the next call resumes)")
    ap.add_argument("--resume-from", default=None, help="--error-run: another directory holding a checkpoint")
    ap.add_argument("--error-summary", metavar="DIR",
                    help="summarise the --error-run results in DIR into profiles/fixed_error_<workload>.json")
    ap.add_argument("--autocorr-json", default=None, help="--error-summary: a saved --autocorr result to include")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-fixed-error", action="store_true",
                    help="skip re-timing the fast form at its equal-error sample count (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run an elementwise device copy of 1 GiB (read 1 GiB, write 1 GiB), the known-size "
                         "reference that scales the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30}))
        return
    if args.error_summary:
        res = error_summary(args.error_summary, args.workload, args.autocorr_json)
        path = os.path.join(ROOT, "profiles", "fixed_error_%s.json" % args.workload)
        with open(path, "w") as f:
            json.dump(res, f, indent=1)
        print(json.dumps({k: res[k] for k in ("n_samples_plain", "e_plain", "n_samples_fast", "e_fast")}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: one GPU only (trajectories shard across GPUs by design, but there is no "
              "multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2506_23928_amd as tv
    import workloads as wl
    if args.workload == "uneven":
        bench_uneven(tv, args)
        return
    w = dict(wl.WORKLOADS[args.workload])
    w["name"] = args.workload
    kind, nh, m, _ = ansatz_of(tv, w)
    prec = tv.PREC_MFMA if args.precision == "mfma" else tv.PREC_FP64
    n, T = w["n"], w["n_traj"]
    print("bench: workload %s N=%d M=%d trajectories=%d samples=%d chains=%d jumps=%d precision=%s proposal=%s" % (
        args.workload, n, m, T, w["n_samples"], w["n_chains"], len(wl.jumps(w)), args.precision,
        w.get("proposal", "flip")), file=sys.stderr, flush=True)

    if args.log:
        from paper_2506_23928_amd.metrics import JsonlLog
        ctx = build_context(tv, w, prec)
        ctx.set_timing(True)
        log = JsonlLog(args.log)
        for _ in range(args.steps):
            ctx.sde_step(1)
            log.write(ctx, workload=args.workload)
        log.close()
        print(json.dumps({"workload": args.workload, "steps": args.steps, "log": args.log}), flush=True)
        return
    if args.error_run:
        parts = args.error_run.split(":")
        error_run(tv, w, parts[0], int(parts[1]), args.out, dt=float(parts[2]) if len(parts) > 2 else None,
                  max_seconds=args.max_seconds, resume_dir=args.resume_from)
        return
    if args.autocorr:
        res = autocorrelation(tv, w, args.steps, min(T, 16))
        print(json.dumps({"workload": args.workload, "steps": args.steps, "samples_per_chain":
                          w["n_samples"] // w["n_chains"], "thin_sweeps": w["thin_sweeps"], **res}), flush=True)
        return
    solver = {"auto": tv.tvmc.SOLVER_AUTO, "one": tv.tvmc.SOLVER_ONE_GROUP, "multi": tv.tvmc.SOLVER_MULTI_GROUP}[args.solver]
    reg = tv.tvmc.REG_SNR if args.regulariser == "snr" else tv.tvmc.REG_SHIFT
    ctx = build_context(tv, w, prec, solver=solver, regulariser=reg, graph=args.graph,
                        sampler_chains=args.sampler_chains)
    for _ in range(args.warmup):
        ctx.sde_step(1)
    ctx.synchronize()
    print("bench: warmup done", file=sys.stderr, flush=True)
    ctx.set_timing(not args.graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.sde_step(1)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.synchronize()
    groups = {}
    for g in ("sample", "estimate", "transpose", "sbuild", "solve", "update", "observe", "train"):
        ms, cnt = ctx.timing(g)
        if cnt:
            groups[g] = {"avg_ms": ms, "launches": cnt, "total_ms": ms * cnt}
    ctx.set_timing(False)
    value = T * args.steps / el
    print("bench: %d steps in %.3f s -> %.1f trajectory-steps/s" % (args.steps, el, value), file=sys.stderr,
          flush=True)

    ss, ns = ctx.sample_space, w["n_samples"]
    roof = roofline_of(tv, groups, kind, prec, ss, m, ns, nh, T, reg, args.solver, n=n)
    # the other heavy groups against their own roofs (the S-build, the operand split, the solve)
    secondary = [r for r in (roofline_of(tv, groups, kind, prec, ss, m, ns, nh, T, reg, args.solver, group=g, n=n)
                             for g in ("sbuild", "solve", "transpose") if g in groups and g != roof["kernel"] and
                             roof["kernel"] not in _KERNELS_OF.get(g, ()))
                 if r["achieved"] is not None]
    del ctx
    torch.cuda.empty_cache()

    # the fixed-xi^2-error protocol's result (profiles/fixed_error_<workload>.json, from --error-run
    # and --error-summary): the fast form's N_s at equal error, timed here over the same steps
    fixed = None
    fe_path = os.path.join(ROOT, "profiles", "fixed_error_%s.json" % args.workload)
    if os.path.exists(fe_path) and not args.graph and not args.no_fixed_error:
        fe = json.load(open(fe_path))
        ns_f = fe["n_samples_fast"]
        rate_f = value
        if ns_f and ns_f != w["n_samples"]:
            wf = dict(w)
            wf["n_samples"] = ns_f
            fctx = build_context(tv, wf, prec, solver=solver, regulariser=reg)
            for _ in range(args.warmup):
                fctx.sde_step(1)
            fctx.synchronize()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                fctx.sde_step(1)
            torch.cuda.synchronize()
            rate_f = T * args.steps / (time.perf_counter() - t1)
            del fctx
            torch.cuda.empty_cache()
            print("bench: fast form at the equal-error N_s = %d: %.1f trajectory-steps/s" % (ns_f, rate_f),
                  file=sys.stderr, flush=True)
        f8 = [r for r in fe["fast"] if r["n_samples"] == w["n_samples"]]
        fixed = {"source": os.path.relpath(fe_path, ROOT), "n_samples_plain": fe["n_samples_plain"],
                 "e_plain": fe["e_plain"], "e_plain_sigma": fe["e_plain_sigma"], "n_samples_fast": ns_f,
                 "e_fast": fe["e_fast"], "e_fast_at_config_n_samples": f8[0]["e"] if f8 else None,
                 "value_fast_at_equal_error": rate_f}

    plain = None
    if not args.no_plain:
        # the plain form: FP64 S-build, one trajectory per launch
        pctx = build_context(tv, w, tv.PREC_FP64, n_traj=1, proposal=tv.PROPOSAL_FLIP)
        pctx.sde_step(1)
        pctx.synchronize()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pctx.sde_step(2)
        torch.cuda.synchronize()
        plain = 2.0 / (time.perf_counter() - t1)
        del pctx
        torch.cuda.empty_cache()
        print("bench: plain form (FP64 S, one trajectory per launch) %.3f trajectory-steps/s" % plain,
              file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, ns_sample=256 if w.get("ansatz") == "rbm" else None, regulariser=reg)

    out = {
        "metric": "trajectory-steps/s at N=64 (batched+learned vs plain) at fixed xi^2 error",
        "value": value, "unit": "trajectory-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if (prec == tv.PREC_FP64 or kind != tv.RBM or ss) else "f64+bf16x3",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_spins": n, "n_params": m, "n_traj": T, "n_samples": w["n_samples"],
                   "n_chains": w["n_chains"], "n_jumps": len(wl.jumps(w)), "dt": w["dt"],
                   "ansatz": w.get("ansatz", "jastrow"), "n_hidden": nh if kind == tv.RBM else 0,
                   **({"ljph_d": nh} if kind == tv.LJPH else {}), "proposal": w.get("proposal", "flip"),
                   "s_build": ("sample-space kernel O O^H (FP64 MFMA Gram)" if kind == tv.RBM else
                               "sample-space kernel O O^H (integer closed form)") if ss else
                   ("int8 MFMA (exact)" if prec == tv.PREC_MFMA else "FP64 VALU") if kind != tv.RBM
                   else ("BF16-split MFMA, FP32 accumulate" if prec == tv.PREC_MFMA else "FP64 VALU (complex)"),
                   "solve": ("FP64 Jacobi + SNR filter (tau %g)" % w.get("snr_tau", 4.0)) if reg == tv.tvmc.REG_SNR
                   else "FP64 Cholesky" + (" (sample space)" if ss else ""), "solver": args.solver,
                   "obs_every": w["obs_every"]},
        "roofline": roof,
        "rooflines_secondary": secondary,
        "cpu_baseline": cpu,
        "plain_form_value": plain,
        "fixed_error": dict(fixed, ratio_at_equal_error=(fixed["value_fast_at_equal_error"] / plain) if plain else None)
        if fixed else None,
        "kernel_ms": {g: round(v["avg_ms"], 4) for g, v in groups.items()},
        "kernel_sources_sha": kernel_sources_sha(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
