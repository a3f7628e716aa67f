"""The benchmark workloads and their end-to-end drivers (set-up, deflation
build, solves, network training), all through the C ABI.

Synthetic inputs stand in for the paper's beta = 5.3 dynamical ensembles on
48 x 24^3 (not available): random SU(3) links exp(i eps H) at the lattice sizes
and hopping parameters below, Gaussian sources.  Seeds: gauge field of workload
i: 1000 + i; sources 2000 + 100 i + r; network training sources 3000+; test
sources 4000+; deflation start fields 5000 + i.
"""
from __future__ import annotations

import os
import time

import numpy as np

from . import qdd
from . import synth as S

WORKLOADS = {
    1: dict(L=(4, 4, 4, 4), eps=0.3, kappa=0.13, csw=1.9, nrhs=1, op="Dhat", precond=qdd.PRECOND_NONE),
    2: dict(L=(32, 16, 16, 16), eps=0.5, kappa=0.1355, csw=1.9, nrhs=12, sap_bs=(4, 4, 4, 4), nmr=4, ncy=5,
            sap_prec=qdd.F32, dfl_Ns=20, precond=qdd.PRECOND_DFL),
    3: dict(L=(64, 32, 32, 32), eps=0.6, kappa=0.1357, csw=1.9, nrhs=8, sap_bs=(4, 4, 4, 4), nmr=4, ncy=5,
            sap_prec=qdd.F16, dfl_Ns=24, precond=qdd.PRECOND_DFL),
    4: dict(lattices=[(8, 8, 8, 8), (16, 16, 16, 16), (48, 24, 24, 24), (64, 32, 32, 32)],
            kappas=[0.1350, 0.1355, 0.1357], eps=0.6, csw=1.9, nrhs=4, sap_bs=(4, 4, 4, 4), nmr=4, ncy=5,
            sap_prec=qdd.F32, dfl_Ns=20, precond=qdd.PRECOND_DFL),
    5: dict(L=(48, 24, 24, 24), eps=0.6, kappa=0.1357, csw=1.9, nrhs=12, sap_bs=(4, 4, 4, 4), nmr=4, ncy=5,
            sap_prec=qdd.F32, dfl_Ns=20, precond=qdd.PRECOND_DFL, net_ch=(1, 12, 12, 1), train_pairs=4096),
}


TUNE_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def make_context(L, eps, kappa, csw, gauge_seed, U=None, tune_nrhs=0, stream=None, **cfg):
    """Context with the gauge field and clover set up; returns (ctx, links).
    tune_nrhs > 0: the Schwarz kernel variant is tuned for that batch size (the
    choice is cached in the package's tuner cache)."""
    import torch

    if U is None:
        U = S.random_su3_links(L, eps, gauge_seed)
    c = qdd.Context(L, qdd.default_config(**cfg), stream=stream)
    c.set_gauge(torch.from_numpy(U))
    c.set_params(kappa, csw)
    if tune_nrhs > 0 and c.cfg.sap_prec != qdd.F64 and c.cfg.precond != qdd.PRECOND_NONE:
        cache = qdd.load_tune_cache(TUNE_CACHE)
        c.tune_sap(tune_nrhs, cache=cache)
        qdd.save_tune_cache(TUNE_CACHE, cache)
    return c, U


def solver_config(w: dict, nrhs: int, plain: bool = False, use_net: bool = False, **extra):
    """qdd_config keywords for a workload; plain = FP64 SAP, FP64 deflation."""
    cfg = dict(max_nrhs=nrhs, sap_bs=w.get("sap_bs", (4, 4, 4, 4)), nmr=w.get("nmr", 4), ncy=w.get("ncy", 5),
               sap_prec=qdd.F64 if plain else w.get("sap_prec", qdd.F32), dfl_Ns=w.get("dfl_Ns", 0),
               dfl_bs=w.get("dfl_bs", (4, 4, 4, 4)), precond=w.get("precond", qdd.PRECOND_NONE))
    if use_net:
        ch = w.get("net_ch", (1, 12, 12, 1))
        cfg.update(use_net=1, net_nl=len(ch) - 1, net_ch=ch)
    cfg.update(extra)
    return cfg


def on_device(a, device="cuda:0"):
    """complex128 device tensor of a host array (the transfer happens here, outside
    every timed region: the timings start with their inputs resident in HBM)."""
    import torch

    t = torch.as_tensor(a).to(device=device, dtype=torch.complex128).contiguous()
    torch.cuda.synchronize()
    return t


def timed_solve(ctx, eta):
    import torch

    eta = on_device(eta, ctx.device)
    torch.cuda.synchronize()
    t0 = time.time()
    psi, info, st = ctx.solve(eta, check=False)
    torch.cuda.synchronize()
    return psi, info, st, time.time() - t0


def run_solve_workload(wid: int, plain_rhs: int = 1, log=print, U=None):
    """Mixed-precision batched deflated solve of workload wid next to the plain
    FP64 solver (one right-hand side, FP64 SAP and deflation).  U: the links of
    the workload if already generated.  Returns a dict."""
    import torch

    w = WORKLOADS[wid]
    L = w["L"]
    V = int(np.prod(L))
    nrhs = w["nrhs"]
    out = {"workload": wid, "lattice": "x".join(map(str, L)), "nrhs": nrhs}
    t0 = time.time()
    if U is None:
        U = S.random_su3_links(L, w["eps"], S.gauge_seed(wid))
    log(f"[w{wid}] links {time.time() - t0:.1f} s")
    eta = np.stack([S.gaussian_field(V, S.source_seed(wid, r)) for r in range(nrhs)])
    init = on_device(S.gaussian_field(V, S.dfl_seed(wid), nrhs=w.get("dfl_Ns", 1)))
    # mixed precision, batched
    ctx, _ = make_context(L, w["eps"], w["kappa"], w["csw"], 0, U=U, tune_nrhs=nrhs, **solver_config(w, nrhs))
    if w.get("dfl_Ns"):
        torch.cuda.synchronize()
        t0 = time.time()
        ctx.dfl_build(init)
        torch.cuda.synchronize()
        out["dfl_build_s"] = time.time() - t0
    psi, info, st, dt = timed_solve(ctx, eta)
    out["mixed"] = {"solve_s": dt, "iters": [i["iters"] for i in info],
                    "true_res_max": max(i["true_res"] for i in info), "converged": all(i["converged"] for i in info),
                    "sap_prec": {0: "f64", 1: "f32", 2: "f16"}[ctx.cfg.sap_prec],
                    "gpu_ms": info[0]["gpu_ms"]}
    log(f"[w{wid}] mixed: {out['mixed']}")
    # Q_S^{-1} (Eq. 5) on fresh even sources through the same solver and subspace
    phi = S.gaussian_field_device(V // 2, 6000, nrhs)
    torch.cuda.synchronize()
    t0 = time.time()
    _, qinfo, _ = ctx.solve_qs(phi, check=False)
    torch.cuda.synchronize()
    out["qs_inverse"] = {"solve_s": time.time() - t0, "iters": [i["iters"] for i in qinfo],
                         "converged": all(i["converged"] for i in qinfo)}
    log(f"[w{wid}] Q_S inverse: {out['qs_inverse']}")
    # the effective action of Eq. 4 with two pseudofermions at dm = 0.09 (the mass
    # difference of the paper's runs): clover log determinants, W^{-1}(dm) phi1 and
    # Q_S^{-1} phi2 as one batch of two solves through the same solver
    if nrhs >= 2:
        ph = S.gaussian_field_device(V // 2, 6100, 2)
        torch.cuda.synchronize()
        t0 = time.time()
        s_eff, parts, _, _, ainfo = ctx.action(0.09, ph[0], ph[1])
        torch.cuda.synchronize()
        out["action_eq4"] = {"dm": 0.09, "s_eff": s_eff, "parts": list(parts), "s": time.time() - t0,
                             "iters": [i["iters"] for i in ainfo], "residuals": [i["true_res"] for i in ainfo]}
        log(f"[w{wid}] action: {out['action_eq4']}")
    del ctx
    torch.cuda.empty_cache()
    if plain_rhs <= 0:
        return out
    # plain FP64 reference solver on plain_rhs right-hand sides, one at a time
    pctx, _ = make_context(L, w["eps"], w["kappa"], w["csw"], 0, U=U, **solver_config(w, 1, plain=True))
    if w.get("dfl_Ns"):
        torch.cuda.synchronize()
        t0 = time.time()
        pctx.dfl_build(init)
        torch.cuda.synchronize()
        out["plain_dfl_build_s"] = time.time() - t0
    ts, its = [], []
    for r in range(plain_rhs):
        _, pinfo, pst, pdt = timed_solve(pctx, eta[r:r + 1])
        ts.append(pdt)
        its.append(pinfo[0]["iters"])
    out["plain_fp64"] = {"solve_s_per_rhs": float(np.mean(ts)), "iters": its, "rhs_timed": plain_rhs}
    out["plain_fp64"]["solve_s_batch_equiv"] = out["plain_fp64"]["solve_s_per_rhs"] * nrhs
    out["speedup_vs_plain"] = out["plain_fp64"]["solve_s_batch_equiv"] / out["mixed"]["solve_s"]
    log(f"[w{wid}] plain: {out['plain_fp64']}")
    del pctx
    torch.cuda.empty_cache()
    return out


def run_learned(wid: int = 5, train_pairs: int | None = None, chunk_pairs: int = 64, batch: int = 4,
                lr: float = 1e-3, epochs: int = 1, test_rhs: int | None = None, harvest_rhs: int | None = None,
                kappa: float | None = None, log=print):
    """Learned preconditioner workload: harvest (r_k, e_k) pairs from plain
    deflated SAP-GCR solves on training sources (harvest_rhs sources per batched
    solve, default the test batch size), train the network on them in streamed
    chunks, then solve fresh test sources with and without the network stage
    (same deflation subspace).  kappa: another hopping parameter on the same
    gauge field (an extra workload closer to the critical one, where the plain
    solver needs more iterations).  Returns a dict."""
    import torch

    w = dict(WORKLOADS[wid])
    if kappa is not None:
        w["kappa"] = kappa
    L = w["L"]
    V = int(np.prod(L))
    ntest = test_rhs or w["nrhs"]
    harvest_rhs = min(harvest_rhs or ntest, ntest)
    npairs = train_pairs or w["train_pairs"]
    out = {"workload": wid, "lattice": "x".join(map(str, L)), "kappa": w["kappa"], "train_pairs_target": npairs}
    U = S.random_su3_links(L, w["eps"], S.gauge_seed(wid))
    init = on_device(S.gaussian_field(V, S.dfl_seed(wid), nrhs=w["dfl_Ns"]))
    ctx, _ = make_context(L, w["eps"], w["kappa"], w["csw"], 0, U=U, tune_nrhs=ntest,
                          **solver_config(w, ntest, use_net=True))
    torch.cuda.synchronize()
    t0 = time.time()
    ctx.dfl_build(init)
    torch.cuda.synchronize()
    out["dfl_build_s"] = time.time() - t0
    nw = ctx.net_num_weights()
    ctx.net_set_weights(S.random_weights(nw, 3000, 0.02))
    # harvest and train in streamed chunks
    rb, eb = ctx.pair_buffers(chunk_pairs)
    fb32 = ctx.field_bytes(qdd.F32, 1, False)
    got, src, steps, losses = 0, 0, 0, []
    t_h = t_t = 0.0
    while got < npairs:
        n_chunk = 0
        t0 = time.time()
        while n_chunk < chunk_pairs and got + n_chunk < npairs:
            # a batch of plain solves; every iteration of every source gives a pair
            eta = S.gaussian_field_device(V, 3000 + src, harvest_rhs)
            src += harvest_rhs
            room = chunk_pairs - n_chunk
            rview = rb[n_chunk * fb32:]
            # the FP32 pairs of earlier batches sit packed at the front of both buffers
            _, info, n, _ = ctx.solve_harvest(eta, rview, eb[n_chunk * fb32:], min(room, npairs - got - n_chunk),
                                              check=False)
            n_chunk += n
        torch.cuda.synchronize()
        t_h += time.time() - t0
        t0 = time.time()
        for _ in range(epochs):
            for b0 in range(0, n_chunk - batch + 1, batch):
                losses.append(ctx.net_train_step(rb[b0 * fb32:], eb[b0 * fb32:], batch, lr))
                steps += 1
        torch.cuda.synchronize()
        t_t += time.time() - t0
        got += n_chunk
        log(f"[w{wid}] pairs {got}/{npairs} solves {src} steps {steps} loss {losses[-1] if losses else None}")
    out.update(train_pairs=got, train_solves=src, train_steps=steps, harvest_s=t_h, train_s=t_t,
               loss_first=losses[0] if losses else None, loss_last=losses[-1] if losses else None)
    # evaluate on fresh sources: learned vs plain (same deflation subspace, network off)
    eta = on_device(np.stack([S.gaussian_field(V, 4000 + r) for r in range(ntest)]))
    psi, info, st, dt = timed_solve(ctx, eta)
    out["learned"] = {"solve_s": dt, "iters": [i["iters"] for i in info], "fallbacks": [i["fallbacks"] for i in info],
                      "true_res_max": max(i["true_res"] for i in info), "converged": all(i["converged"] for i in info),
                      "t_ms": info[0]["t_ms"], "gpu_ms": info[0]["gpu_ms"]}
    # the same network applied with activations rounded to one BF16 term (8
    # significant bits) in its products: a cheaper, inexact preconditioner stage
    ctx.net_set_terms(1)
    psi, info, st, dt = timed_solve(ctx, eta)
    out["learned_terms1"] = {"solve_s": dt, "iters": [i["iters"] for i in info],
                             "fallbacks": [i["fallbacks"] for i in info],
                             "true_res_max": max(i["true_res"] for i in info),
                             "converged": all(i["converged"] for i in info), "t_ms": info[0]["t_ms"]}
    # the network stage only in the first 1 or 2 outer iterations of the solve
    for calls in (1, 2):
        ctx.net_set_calls(calls)
        for terms in (3, 1):
            ctx.net_set_terms(terms)
            psi, info, st, dt = timed_solve(ctx, eta)
            out[f"learned_calls{calls}_terms{terms}"] = {
                "solve_s": dt, "iters": [i["iters"] for i in info], "fallbacks": [i["fallbacks"] for i in info],
                "true_res_max": max(i["true_res"] for i in info), "converged": all(i["converged"] for i in info)}
    ctx.net_set_calls(0)
    ctx.net_set_terms(3)
    ctx.net_set_weights(np.zeros(nw, complex))  # zero network: the stage adds nothing, plain iterates
    psi0, info0, st0, dt0 = timed_solve(ctx, eta)
    out["plain_same_subspace"] = {"solve_s": dt0, "iters": [i["iters"] for i in info0],
                                  "true_res_max": max(i["true_res"] for i in info0)}
    del ctx
    torch.cuda.empty_cache()
    # plain method proper: no network stage at all
    pctx, _ = make_context(L, w["eps"], w["kappa"], w["csw"], 0, U=U, tune_nrhs=ntest, **solver_config(w, ntest))
    pctx.dfl_build(init)
    psi1, info1, st1, dt1 = timed_solve(pctx, eta)
    out["plain"] = {"solve_s": dt1, "iters": [i["iters"] for i in info1],
                    "true_res_max": max(i["true_res"] for i in info1), "t_ms": info1[0]["t_ms"],
                    "gpu_ms": info1[0]["gpu_ms"]}
    out["learned_vs_plain_time"] = dt1 / out["learned"]["solve_s"]
    log(f"[w{wid}] learned {out['learned']} plain {out['plain']}")
    return out


def run_multi(wid: int = 4, nkv: int = 8, precond: str = "sap", modes=None, log=print):
    """Batched uneven solves: every lattice of the workload at every mass, nrhs
    right-hand sides each.  precond "sap": FP32 Schwarz preconditioner, no
    deflation; the systems are solved (1) as one group, every solver stage one
    launch over all systems (qdd_solve_group), (2) concurrently on their own
    streams from host threads (qdd_solve_multi) and (3) one after the other.
    precond "dfl": the deflated solver (subspace built once per lattice at the
    middle mass and shared with the other masses), modes (2) and (3).  The
    Schwarz kernel variant tuned for the largest lattice is used by all systems.
    modes: a subset of the modes to run (the equality checks against the
    sequential solve need "sequential").  Returns a dict."""
    import torch

    w = WORKLOADS[wid]
    nrhs = w["nrhs"]
    dfl = precond == "dfl"
    ctxs, etas, names = [], [], []
    t_setup = time.time()
    t_build = 0.0
    extra = dict(nkv=nkv) if dfl else dict(nkv=nkv, precond=qdd.PRECOND_SAP, dfl_Ns=0)
    for li, L in enumerate(w["lattices"]):
        V = int(np.prod(L))
        U = S.random_su3_links(L, w["eps"], S.gauge_seed(wid) + 10 * li)
        group = []
        for ki, kappa in enumerate(w["kappas"]):
            c, _ = make_context(L, w["eps"], kappa, w["csw"], 0, U=U, tune_nrhs=nrhs, stream=torch.cuda.Stream(),
                                **solver_config(w, nrhs, **extra))
            group.append(c)
            etas.append(on_device(np.stack([S.gaussian_field(V, S.source_seed(wid, 10 * li + r) + ki)
                                            for r in range(nrhs)])))
            names.append(f"{'x'.join(map(str, L))}/k{kappa}")
        if dfl:
            init = on_device(S.gaussian_field(V, S.dfl_seed(wid) + 10 * li, nrhs=w["dfl_Ns"]))
            mid = len(group) // 2
            torch.cuda.synchronize()
            t0 = time.time()
            group[mid].dfl_build(init)
            for k, c in enumerate(group):
                if k != mid:
                    c.dfl_share(group[mid])
            torch.cuda.synchronize()
            t_build += time.time() - t0
        ctxs += group
        del U
        log(f"[w{wid}] lattice {L} ready")
    big = max(range(len(ctxs)), key=lambda k: ctxs[k].V)
    variant = ctxs[big].get_launch(qdd.KERNEL_SAP, w["sap_prec"])[1]
    for c in ctxs:
        c.set_launch(qdd.KERNEL_SAP, w["sap_prec"], 0, variant, 0, 0)
    out = {"workload": wid, "precond": precond, "systems": len(ctxs), "nrhs_each": nrhs,
           "setup_s": time.time() - t_setup, "sap_variant": variant}
    if dfl:
        out["dfl_build_s"] = t_build

    def record(key, psis, infos, st, dt):
        out[key + "_s"] = dt
        out[key + "_status"] = st
        out[key + "_systems"] = [{"system": n, "iters": [i["iters"] for i in inf],
                                  "converged": all(i["converged"] for i in inf),
                                  "true_res_max": max(i["true_res"] for i in inf)} for n, inf in zip(names, infos)]

    def solve(mode):
        if mode == "sequential":
            psis, infos, st = [], [], 0
            for c, eta in zip(ctxs, etas):
                p, i, s1 = c.solve(eta, check=False)
                torch.cuda.synchronize()
                psis.append(p)
                infos.append(i)
                st = st or s1
            return psis, infos, st
        if mode == "threads":
            return qdd.solve_multi(ctxs, etas)
        return qdd.solve_group(ctxs, etas)

    results = {}
    modes = [m for m in (["threads", "sequential"] if dfl else ["group", "threads", "sequential"])
             if modes is None or m in modes]
    for mode in modes:
        # the second of two runs is timed (the first loads the kernels it uses)
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.time()
            psis, infos, st = solve(mode)
            torch.cuda.synchronize()
            dt = time.time() - t0
        record(mode, psis, infos, st, dt)
        results[mode] = psis
        log(f"[w{wid}] {precond} {mode}: {out[mode + '_s']:.3f} s status {st}")
    if "sequential" in results:
        seq = results["sequential"]
        for mode in results:
            if mode != "sequential":
                out[mode + "_equals_sequential"] = all(torch.equal(a, b) for a, b in zip(results[mode], seq))
    out["all_converged"] = all(d["converged"] for m in modes for d in out[m + "_systems"])
    out["true_res_max"] = max(d["true_res_max"] for m in modes for d in out[m + "_systems"])
    return out


def run_block_solve(wid: int = 5, bs=(12, 12, 6, 6), nrhs: int = 2, tol: float = 1e-10, U=None, log=print):
    """Dirichlet block solves of the DD-HMC forces (BiCGstab on every block, one
    launch) on the lattice and field of workload wid with blocks of extent bs
    (the paper's 6^2 x 12^2 blocks of the 48 x 24^3 lattice), nrhs Gaussian
    sources.  Model bytes per iteration and even site: two block Dhat at the
    2-pass model (4416 B in FP64) plus 16 FP64 vector passes (192 B each); the
    rate divides the iterations every block took by the GPU time of the launch.
    Returns a dict."""
    import torch

    w = WORKLOADS[wid]
    L = w["L"]
    V = int(np.prod(L))
    if U is None:
        U = S.random_su3_links(L, w["eps"], S.gauge_seed(wid))
    ctx = qdd.Context(L, qdd.default_config(max_nrhs=nrhs, blk_bs=bs))
    ctx.set_gauge(torch.from_numpy(U))
    ctx.set_params(w["kappa"], w["csw"])
    eta = torch.from_numpy(np.stack([S.gaussian_field(V, S.source_seed(wid, 50 + r)) for r in range(nrhs)])).cuda()
    ctx.block_solve(eta, tol=tol)  # first call also gathers links and clover into the block-major layout
    torch.cuda.synchronize()
    t0 = time.time()
    _, it, res, info, st = ctx.block_solve(eta, tol=tol, check=False)
    torch.cuda.synchronize()
    wall = time.time() - t0
    neb = V // 2 // info["nblk"] * nrhs
    per_iter = 2 * 4416 + 16 * 192
    model = float(it.clamp(min=0).sum()) * neb * per_iter
    out = {"lattice": "x".join(map(str, L)), "block": "x".join(map(str, bs)), "blocks": info["nblk"] // nrhs,
           "nrhs": nrhs, "tol": tol, "kernel_ms": info["t_ms"], "wall_s": wall, "iters_min": int(it.min()),
           "iters_max": int(it.max()), "res_max": info["res_max"], "converged": info["converged"] == info["nblk"],
           "model_bytes": model, "model_TBs": model / (info["t_ms"] * 1e-3) / 1e12, "status": st}
    log(f"[blk] {out}")
    del ctx
    torch.cuda.empty_cache()
    return out


def time_network(wid: int = 5, reps: int = 5, nb: int = 4, log=print):
    """Timing of the learned stage's kernels on the workload lattice: one
    forward pass of the network on a Gaussian field and one Adam training step
    on nb random pairs (mean over reps, after one warm-up each); the forward
    also with one and two BF16 terms per activation.  Returns a dict."""
    import torch

    w = WORKLOADS[wid]
    L = w["L"]
    V = int(np.prod(L))
    U = S.random_su3_links(L, w["eps"], S.gauge_seed(wid))
    ctx, _ = make_context(L, w["eps"], w["kappa"], w["csw"], 0, U=U, **solver_config(w, 1, use_net=True))
    ctx.net_set_weights(S.random_weights(ctx.net_num_weights(), 3000, 0.05))
    x = S.gaussian_field_device(V, 5000, 1)[0]
    fwd_t = {}
    for terms in (1, 2, 3):
        ctx.net_set_terms(terms)
        ctx.net_forward(x)
        torch.cuda.synchronize()
        t0 = time.time()
        for _ in range(reps):
            ctx.net_forward(x)
        torch.cuda.synchronize()
        fwd_t[terms] = (time.time() - t0) / reps
    fwd = fwd_t[3]
    rb, eb = ctx.pair_buffers(nb)
    fb32 = ctx.field_bytes(qdd.F32, 1, False)
    for k in range(nb):  # FP32 pairs: random residuals and errors
        for buf, seed in ((rb, 6000 + k), (eb, 7000 + k)):
            buf[k * fb32:(k + 1) * fb32].view(torch.float32).copy_(
                torch.view_as_real(S.gaussian_field_device(V, seed, 1)).flatten().to(torch.float32))
    ctx.net_train_step(rb, eb, nb, 1e-4)
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(reps):
        ctx.net_train_step(rb, eb, nb, 1e-4)
    torch.cuda.synchronize()
    out = {"lattice": "x".join(map(str, L)), "channels": list(w.get("net_ch", (1, 12, 12, 1))),
           "forward_ms": fwd * 1e3, "forward_ms_terms2": fwd_t[2] * 1e3, "forward_ms_terms1": fwd_t[1] * 1e3,
           "train_step_ms": (time.time() - t0) / reps * 1e3, "pairs_per_step": nb}
    log(f"[net] {out}")
    return out


def time_sap(L=(64, 32, 32, 32), prec=qdd.F16, nrhs=8, reps=3, log=print):
    """Every Schwarz half-sweep kernel variant on one lattice (random links
    exp(i 0.6 H), kappa 0.1357, c_sw 1.9, 4^4 blocks, nmr 4, ncy 5): mean wall time
    of reps preconditioner calls M_sap on nrhs Gaussian sources (canonical fields
    in and out, so packing included).  Returns a dict; run it under rocprofv3 for
    the per-kernel times."""
    import torch

    V = int(np.prod(L))
    ctx, _ = make_context(L, 0.6, 0.1357, 1.9, S.gauge_seed(3) if L == (64, 32, 32, 32) else 1600,
                          max_nrhs=nrhs, sap_prec=prec, precond=qdd.PRECOND_SAP, nkv=1)
    eta = S.gaussian_field_device(V, 77, nrhs)
    out = {"lattice": "x".join(map(str, L)), "prec": prec, "nrhs": nrhs, "ms_per_call": {}}
    for v in ((1, 2, 3, 4) if prec == qdd.F16 else (1, 2, 3)):
        ctx.set_launch(qdd.KERNEL_SAP, prec, 0, v, 0, 0)
        ctx.sap(eta)
        torch.cuda.synchronize()
        t0 = time.time()
        for _ in range(reps):
            ctx.sap(eta)
        torch.cuda.synchronize()
        out["ms_per_call"][v] = (time.time() - t0) / reps * 1e3
        log(f"[sap] variant {v}: {out['ms_per_call'][v]:.1f} ms per call")
    return out


def main(argv=None):
    """Command line: python -m paper_1011_0911_amd.workloads WID [--pairs N]
    runs one workload driver on cuda:0 and prints its result as one JSON line;
    WID = net times the network forward pass and a training step on the
    workload-5 lattice, WID = sap every Schwarz kernel variant on the workload-3
    lattice (FP16 storage, 8 right-hand sides)."""
    import argparse
    import json

    ap = argparse.ArgumentParser()
    ap.add_argument("wid", choices=["2", "3", "4", "5", "net", "sap"])
    ap.add_argument("--pairs", type=int, default=None, help="training pairs (workload 5)")
    ap.add_argument("--chunk", type=int, default=64, help="pairs per streamed training chunk (workload 5)")
    ap.add_argument("--epochs", type=int, default=1)
    ap.add_argument("--kappa", type=float, default=None, help="workload 5: hopping parameter instead of 0.1357")
    ap.add_argument("--precond", choices=["sap", "dfl"], default="sap", help="workload 4: preconditioner")
    ap.add_argument("--modes", default=None, help="workload 4: comma-separated subset of group,threads,sequential")
    ap.add_argument("--sap-prec", type=int, default=qdd.F16, help="sap: storage precision (1 FP32, 2 FP16)")
    ap.add_argument("--nrhs", type=int, default=8, help="sap: right-hand sides")
    ap.add_argument("--plain-rhs", type=int, default=1,
                    help="right-hand sides timed with the plain solver (0: mixed solver only)")
    a = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)  # noqa: E731
    if a.wid == "net":
        r = time_network(5, log=log)
    elif a.wid == "sap":
        r = time_sap(prec=a.sap_prec, nrhs=a.nrhs, log=log)
    elif a.wid == "5":
        r = run_learned(5, train_pairs=a.pairs, chunk_pairs=a.chunk, epochs=a.epochs, kappa=a.kappa, log=log)
    elif a.wid == "4":
        r = run_multi(4, precond=a.precond, modes=a.modes.split(",") if a.modes else None, log=log)
    else:
        r = run_solve_workload(int(a.wid), plain_rhs=a.plain_rhs, log=log)
    print(json.dumps(r, default=float), flush=True)


if __name__ == "__main__":
    main()
