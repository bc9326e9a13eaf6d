"""Benchmark of the animated-octree feature renderer on one MI355X.

One step = one whole-batch render of the full-size workload: FP64 bone chain
-> skinning of 1.5M leaves -> posed-octree rebuild -> ray indexing and
front-to-back compositing into 16-channel feature maps + opacity, for 30 poses
x 8 ring cameras at 512x512 (62.9M rays).  Inputs are seeded synthetic
animal-shaped octrees already resident in HBM when the timed region starts.

Prints one JSON line with Mrays/s, the compositing kernel's fraction of the
HBM roofline (HIP-event timing of every render launch inside the timed region)
and the FP64 CPU oracle timed on a bounded sample on the host.

    python bench.py [--steps K] [--warmup W] [--config full] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_render_full_traffic.txt")
RENDER_SOURCES = ("render_impl.h", "render_c16.hip", "device_util.h", "internal.h")


def render_source_hash():
    """SHA-256 over the sources the compositing kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for f in RENDER_SOURCES:
        with open(os.path.join(ROOT, "paper_2202_05628_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per compositing launch from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel factor), or
    None when the summary is missing, covers another workload or was taken on
    a different version of the kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("render_source_hash") != render_source_hash() or kv.get("workload") != workload:
        return None
    try:
        return int(float(kv["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def copy_probe(torch, nbytes=1 << 30, reps=5):
    """Device-to-device copy bandwidth (read + write bytes / time) of one
    torch copy kernel over nbytes, timed with events on the current stream.
    Run only with --copy-probe: the profiling runs use this copy of known size
    to scale the FETCH_SIZE / WRITE_SIZE counters to bytes.  It is not a
    bound of the compositing kernel (a gather of rows that partly hit in the
    caches), so the record does not compare the kernel with it."""
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    y.copy_(x)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    del x, y
    return 2 * nbytes / s / 1e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="full")
    ap.add_argument("--poses", type=int, default=0, help="override the pose count (profiling)")
    ap.add_argument("--lambda-th", type=float, default=0.01)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-proposal", action="store_true", help="skip the learned-proposal comparison")
    ap.add_argument("--proposal-steps", type=int, default=3)
    ap.add_argument("--train-steps", type=int, default=5000)
    ap.add_argument("--train-rays", type=int, default=4_000_000)
    ap.add_argument("--margin-h", type=float, default=0.0,
                    help="proposal start margin in leaf edges (0: calibrated on held-out rays)")
    ap.add_argument("--f2-tau", type=float, default=-1.0)
    ap.add_argument("--proposal-loss", choices=["smooth_l1", "pinball"], default="pinball",
                    help="training loss of the proposal network (pinball: one-sided interval)")
    ap.add_argument("--tau-near", type=float, default=0.03, help="pinball level of u_near")
    ap.add_argument("--tau-far", type=float, default=0.97, help="pinball level of u_far")
    ap.add_argument("--margin-quantile", type=float, default=0.99,
                    help="quantile of the held-out late starts that the start margin covers")
    ap.add_argument("--err-poses", type=int, default=4, help="poses on which the proposal error is measured")
    ap.add_argument("--no-forms", action="store_true", help="skip the BF16-storage and adjoint legs")
    ap.add_argument("--copy-probe", action="store_true",
                    help="time a 1 GiB device copy (the counter scale of the profiling runs)")
    ap.add_argument("--leg", choices=["bf16", "adjoint", "adjoint_main", "train", "proposal"], default=None,
                    help="run only this form and print its record (profiling)")
    return ap.parse_args()


def written_rays(stats, W):
    """Rays whose output maps the compositing kernel writes: every ray of the
    call when its waves also write the background pixels (tiles with no
    brick; the library's default for maps whose width is a multiple of 4),
    else the rays of the tiles it renders (the background kernel writes the
    rest)."""
    fused = os.environ.get("ARTEMIS_BG_KERNEL") != "1" and W % 4 == 0
    return stats["rays"] if fused else stats["tile_rays"]


def algorithmic_bytes(stats, C, es, W, with_tfinal=True):
    """Bytes the compositing kernel must move: per composited sample the
    density, the C features and the 4-byte leaf-index word; per ray it
    writes the C + 1 output floats (+ the final transmittance)."""
    per_sample = es * (C + 1) + 4
    per_ray = 4 * (C + 1) + (4 if with_tfinal else 0)
    return stats["samples"] * per_sample + written_rays(stats, W) * per_ray


def cpu_baseline(scene, poses, K, c2w, H, W, lam, budget_s):
    """FP64 oracle on the host: one pose built in full (FK, skinning, occupancy),
    its rays rendered on a uniform sample sized to the time budget, the render
    time extrapolated to all rays of the pose."""
    import numpy as np

    import oracle

    oracle.build(force=False)
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    B = oracle.fk(scene.parent, scene.rest_joint, poses[0][:1], poses[1][:1], poses[2][:1])[0]
    ok, ol, _, _, _ = oracle.pose_occupancy(scene.ijk, scene.depth, scene.bone, scene.weight, B)
    t_build = time.perf_counter() - t0
    o, d = oracle.camera_rays(K, c2w, H, W)
    o = o.reshape(-1, 3)
    d = d.reshape(-1, 3)
    n_all = o.shape[0]
    rng = np.random.default_rng(7)
    # calibrate on a small sample, then size the main sample to the budget
    n = 2000
    idx = rng.choice(n_all, n, replace=False)
    t1 = time.perf_counter()
    oracle.render(o[idx], d[idx], scene.depth, ok, ol, scene.sigma, scene.feat, lam)
    rate = n / max(time.perf_counter() - t1, 1e-6)
    n = int(min(n_all, max(2000, rate * max(1.0, budget_s - t_build))))
    idx = rng.choice(n_all, n, replace=False)
    t1 = time.perf_counter()
    oracle.render(o[idx], d[idx], scene.depth, ok, ol, scene.sigma, scene.feat, lam)
    t_render = time.perf_counter() - t1
    t_pose = t_build + t_render * (n_all / n)
    # the render on one host thread, on a sample of about 2 s
    n1 = int(min(n_all, max(500, 2.0 * rate / max(threads, 1))))
    idx = rng.choice(n_all, n1, replace=False)
    t1 = time.perf_counter()
    oracle.render(o[idx], d[idx], scene.depth, ok, ol, scene.sigma, scene.feat, lam, n_threads=1)
    t_one = time.perf_counter() - t1
    return {
        "value": n_all / t_pose / 1e6,
        "unit": "Mrays/s",
        "cores": threads,
        "cpu_model": cpu_model(),
        "host_cpus": os.cpu_count(),
        "kind": "oracle",
        "sample": (f"1 pose x {K.shape[0]} views at {H}x{W}: FK, skinning and occupancy of all "
                   f"{scene.n} leaves timed in full ({t_build:.2f} s); {n} of {n_all} rays rendered "
                   f"({t_render:.2f} s, uniform seeded sample) and extrapolated to the pose"),
        "one_core_render_mrays_s": n1 / t_one / 1e6,
        "one_core_sample": f"{n1} rays of the same pose on one host thread ({t_one:.2f} s)",
    }


def cpu_other_configs(sg, scene, lam, seconds=2.0):
    """The FP64 oracle (all host threads) on the other plain-render workloads:
    the tiny scene (1 pose x 1 camera at 128^2) in full, and one pose of the
    precision-form (16 cameras at 1024^2, BF16-rounded FLUT) and
    learned-proposal (the same cameras, the proposal workload's first pose)
    workloads: FK, skinning and occupancy in full, a seeded uniform ray sample
    of about `seconds`, extrapolated to the pose."""
    import numpy as np

    import oracle

    out = []
    cfg = sg.CONFIGS["tiny"]
    st = sg.make_scene(cfg)
    pt = sg.make_poses(st.J, 1, cfg.pose_seed0)
    Kt, ct = sg.make_cameras(st, cfg.n_views, cfg.height, cfg.width)
    t0 = time.perf_counter()
    B = oracle.fk(st.parent, st.rest_joint, *pt)[0]
    ok, ol, _, _, _ = oracle.pose_occupancy(st.ijk, st.depth, st.bone, st.weight, B)
    o, d = oracle.camera_rays(Kt, ct, cfg.height, cfg.width)
    oracle.render(o.reshape(-1, 3), d.reshape(-1, 3), st.depth, ok, ol, st.sigma, st.feat, lam)
    t = time.perf_counter() - t0
    n_all = cfg.n_views * cfg.height * cfg.width
    out.append({"workload": f"tiny: depth {cfg.depth}, {st.n} leaves, C = {cfg.C}, 1 pose x {cfg.n_views} camera at "
                            f"{cfg.height}x{cfg.width}", "value": n_all / t / 1e6, "unit": "Mrays/s",
                "sample": f"in full ({n_all} rays, FK, skinning and occupancy included, {t:.3f} s)"})
    rng = np.random.default_rng(17)
    for name in ("bf16", "proposal"):
        cfg = sg.CONFIGS[name]
        sig, feat = scene.sigma, scene.feat
        if cfg.storage == "bf16":   # the values the precision form stores
            import torch
            sig = torch.from_numpy(sig).to(torch.bfloat16).float().numpy()
            feat = torch.from_numpy(feat).to(torch.bfloat16).float().numpy()
        p = sg.make_poses(scene.J, 1, cfg.pose_seed0)
        K, c2w = sg.make_cameras(scene, cfg.n_views, cfg.height, cfg.width)
        t0 = time.perf_counter()
        B = oracle.fk(scene.parent, scene.rest_joint, *p)[0]
        ok, ol, _, _, _ = oracle.pose_occupancy(scene.ijk, scene.depth, scene.bone, scene.weight, B)
        t_build = time.perf_counter() - t0
        o, d = oracle.camera_rays(K, c2w, cfg.height, cfg.width)
        o = o.reshape(-1, 3)
        d = d.reshape(-1, 3)
        n_all = o.shape[0]
        idx = rng.choice(n_all, 4000, replace=False)
        t1 = time.perf_counter()
        oracle.render(o[idx], d[idx], scene.depth, ok, ol, sig, feat, lam)
        rate = 4000 / max(time.perf_counter() - t1, 1e-6)
        n = int(min(n_all, max(4000, rate * seconds)))
        idx = rng.choice(n_all, n, replace=False)
        t1 = time.perf_counter()
        oracle.render(o[idx], d[idx], scene.depth, ok, ol, sig, feat, lam)
        t_render = time.perf_counter() - t1
        t_pose = t_build + t_render * (n_all / n)
        out.append({"workload": f"{name}: {cfg.n_poses} poses x {cfg.n_views} cameras at {cfg.height}x{cfg.width}"
                                + (" (BF16-rounded FLUT)" if cfg.storage == "bf16" else ""),
                    "value": n_all / t_pose / 1e6, "unit": "Mrays/s",
                    "sample": f"1 pose: build in full ({t_build:.2f} s); {n} of {n_all} rays ({100.0 * n / n_all:.2f} %, "
                              f"{t_render:.2f} s, uniform seeded sample) extrapolated to the pose; "
                              f"the other poses cost the same"})
    return out


def cpu_model():
    """Model name of the host CPU (first entry of /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_checks(art, sg, torch, lam, n_grad_rays=4000, pixels_per_map=120, bf16_poses=(0, 29)):
    """Errors of the extra forms against the FP64 oracle (part of the CPU-oracle
    leg, the only leg that runs the oracle):

    * precision form: per (pose, view) map of poses `bf16_poses` of the BF16
      workload, rel_max = max|F - F_ref| / max|F_ref| and rel_mean =
      sum|F - F_ref| / sum|F_ref| over sampled pixels (3/4 of them from pixels
      with a sample), against the oracle on the unrounded FP32 FLUT (the whole
      error of the form) and on the BF16-rounded FLUT (arithmetic and FP32
      geometry only); rel_max also outside the rounding guard band (pixels
      whose ray crosses a cell that a leaf within 1e-4 h of a lattice plane
      may land in, where FP32 skinning may place it differently);
    * adjoint: the gradient of L = 1/2 sum (F - F*)^2 over a seeded subset of
      rays of the differentiation workload (dL/dF zero elsewhere), GPU adjoint
      vs the oracle's adjoint over every leaf (rel_max of dsigma and df)."""
    import itertools
    import numpy as np

    import oracle
    out = {}
    # ---- precision form ------------------------------------------------------------
    cfg = sg.CONFIGS["bf16"]
    s = sg.make_scene(cfg)
    r_, R_, T_ = sg.make_poses(s.J, cfg.n_poses, cfg.pose_seed0)
    sel = list(bf16_poses)
    H, W = cfg.height, cfg.width
    K, c2w = sg.make_cameras(s, cfg.n_views, H, W)
    rend = art.Renderer(0)
    rend.set_scene(s)
    rend.set_poses(r_[sel], R_[sel], T_[sel])
    rend.set_cameras(K, c2w, H, W)
    F, A, _ = rend.render(torch.from_numpy(s.sigma).cuda().to(torch.bfloat16),
                          torch.from_numpy(s.feat).cuda().to(torch.bfloat16), lam, fp32_geom=True,
                          want_tfinal=False)
    F = F.cpu().numpy()
    A = A.cpu().numpy()
    rend.close()
    sig_r, feat_r = oracle.bf16_round(s.sigma), oracle.bf16_round(s.feat)
    o, d = oracle.camera_rays(K, c2w, H, W)
    h = 1.0 / (1 << s.depth)
    G = 1 << (s.depth + 1)
    rng = np.random.default_rng(77)
    B = oracle.fk(s.parent, s.rest_joint, r_[sel], R_[sel], T_[sel])
    maps = []
    for pi in range(len(sel)):
        pt = oracle.lbs(s.ijk, s.depth, s.bone, s.weight, B[pi])
        cells, valid = oracle.posed_cells(pt, s.depth)
        ok_, ol_ = oracle.occupancy_from_cells(cells, valid, s.depth)
        u = (pt + 1.0) * (1 << s.depth)
        k = np.round(u)
        near = np.abs(u - k) < 1e-4
        amb = set()
        for i in np.flatnonzero(near.any(axis=1)):
            opts = [(int(k[i, a]) - 1, int(k[i, a])) if near[i, a] else (int(np.floor(u[i, a])),) for a in range(3)]
            amb.update((z * G + y) * G + x for x, y, z in itertools.product(*opts))
        amb_lin = np.array(sorted(amb), dtype=np.int64)
        for v in range(cfg.n_views):
            hitpix = np.flatnonzero(A[pi, v].reshape(-1) > 0)
            nh = min(len(hitpix), pixels_per_map * 3 // 4)
            pix = np.concatenate([rng.choice(hitpix, nh, replace=False),
                                  rng.integers(0, H * W, pixels_per_map - nh)])
            ov, dv = o[v].reshape(-1, 3)[pix], d[v].reshape(-1, 3)[pix]
            ref_a = oracle.render(ov, dv, s.depth, ok_, ol_, s.sigma, s.feat, lam)
            ref_b = oracle.render(ov, dv, s.depth, ok_, ol_, sig_r, feat_r, lam)
            band = ref_a["min_gap"] < 1e-4 * h
            if len(amb_lin):
                band |= oracle.render(ov, dv, s.depth, amb_lin, np.zeros(len(amb_lin), dtype=np.int64),
                                      np.zeros(1), np.zeros((1, 1)), 0.0)["n_hit"] > 0
            Fg = F[pi, v].reshape(s.C, -1)[:, pix]
            row = {"pose": sel[pi], "view": v, "pixels": int(len(pix)), "in_guard_band": int(band.sum())}
            for name, ref in (("total", ref_a), ("arith", ref_b)):
                Fr = ref["F"].T
                err = np.abs(Fg - Fr)
                row[f"{name}_rel_max"] = float(err.max() / np.abs(Fr).max())
                row[f"{name}_rel_max_outside_band"] = float(err[:, ~band].max() / np.abs(Fr[:, ~band]).max())
                row[f"{name}_rel_mean"] = float(err.sum() / np.abs(Fr).sum())
            maps.append(row)
    keys = [k for k in maps[0] if k.endswith(("rel_max", "rel_mean", "outside_band"))]
    out["bf16_form"] = {
        "reference": "FP64 oracle; total = vs the FP32 FLUT, arith = vs the BF16-rounded FLUT",
        "poses": sel, "views": cfg.n_views, "pixels_per_map": pixels_per_map,
        "worst_over_maps": {k: max(m[k] for m in maps) for k in keys},
        "mean_over_maps": {k: float(np.mean([m[k] for m in maps])) for k in keys},
        "maps": maps,
    }
    # ---- adjoint --------------------------------------------------------------------
    cfg = sg.CONFIGS["grad"]
    s = sg.make_scene(cfg)
    poses = sg.make_poses(s.J, cfg.n_poses, cfg.pose_seed0)
    H, W, V = cfg.height, cfg.width, cfg.n_views
    K, c2w = sg.make_cameras(s, V, H, W)
    rend = art.Renderer(0)
    rend.set_scene(s)
    rend.set_poses(*poses)
    rend.set_cameras(K, c2w, H, W)
    B = oracle.fk(s.parent, s.rest_joint, *poses)
    ok_, ol_, _, _, _ = oracle.pose_occupancy(s.ijk, s.depth, s.bone, s.weight, B[0])
    o, d = oracle.camera_rays(K, c2w, H, W)
    o, d = o.reshape(-1, 3), d.reshape(-1, 3)
    tgt = sg.make_targets(1, V, s.C, H, W, seed=cfg.target_seed)[0]
    tgt_rays = np.moveaxis(tgt.reshape(V, s.C, H * W), 1, 2).reshape(-1, s.C)
    rng = np.random.default_rng(1001)
    cand = rng.choice(V * H * W, 6 * n_grad_rays, replace=False)
    ref = oracle.render(o[cand], d[cand], s.depth, ok_, ol_, s.sigma, s.feat, lam)
    good = (ref["min_gap"] >= 1e-9 * h) & (ref["min_tgap"] >= 1e-5)   # away from the rounding guard bands
    hit = good & (ref["n_comp"] > 0)
    sub = np.sort(cand[hit][:n_grad_rays])
    sig = torch.from_numpy(s.sigma).cuda()
    ft = torch.from_numpy(s.feat).cuda()
    Fm, _, Tm = rend.render(sig, ft, lam)
    Fr = Fm[0].permute(0, 2, 3, 1).reshape(-1, s.C)
    g = torch.zeros_like(Fr)
    idx = torch.from_numpy(sub).cuda()
    g[idx] = Fr[idx] - torch.from_numpy(tgt_rays[sub]).cuda()
    dF = g.reshape(1, V, H, W, s.C).permute(0, 1, 4, 2, 3).contiguous()
    ds, df = rend.backward(sig, ft, Fm, Tm, dF, None, lam, reuse_build=True)
    ds = ds.cpu().numpy().astype(np.float64)
    df = df.cpu().numpy().astype(np.float64)
    rend.close()
    refs = oracle.render(o[sub], d[sub], s.depth, ok_, ol_, s.sigma, s.feat, lam)
    ds_ref, df_ref = oracle.backward(o[sub], d[sub], s.depth, ok_, ol_, s.sigma, s.feat, lam,
                                     refs["F"] - tgt_rays[sub])
    out["adjoint_form"] = {
        "reference": "FP64 oracle adjoint, L = 1/2 sum (F - F*)^2 over a seeded subset of rays",
        "rays_in_loss": int(len(sub)), "leaves_with_gradient": int((ds_ref != 0).sum()),
        "dsigma_rel_max": float(np.abs(ds - ds_ref).max() / np.abs(ds_ref).max()),
        "dfeat_rel_max": float(np.abs(df - df_ref).max() / np.abs(df_ref).max()),
    }
    return out


def _timed(torch, fn, steps):
    """Wall time per call of `fn` over `steps` calls after one warm-up call,
    bracketed by device synchronisation."""
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def bf16_leg(args, art, sg, torch):
    """Precision form: BF16 leaf storage, FP32 geometry and accumulation, FP64
    bone chain; 30 poses x 16 cameras at 1024^2 (its errors against the FP64
    oracle are measured by the parity tests)."""
    cfg = sg.CONFIGS["bf16"]
    scene = sg.make_scene(cfg)
    P, V, H, W = cfg.n_poses, cfg.n_views, cfg.height, cfg.width
    r = art.Renderer(0)
    r.set_scene(scene)
    r.set_poses(*sg.make_poses(scene.J, P, cfg.pose_seed0))
    r.set_cameras(*sg.make_cameras(scene, V, H, W), H, W)
    sig = torch.from_numpy(scene.sigma).cuda().to(torch.bfloat16)
    feat = torch.from_numpy(scene.feat).cuda().to(torch.bfloat16)
    F = torch.empty((P, V, cfg.C, H, W), dtype=torch.float32, device="cuda")
    A = torch.empty((P, V, H, W), dtype=torch.float32, device="cuda")
    out = (F, A, None)
    t = _timed(torch, lambda: r.render(sig, feat, args.lambda_th, fp32_geom=True, out=out), args.proposal_steps)
    r.render(sig, feat, args.lambda_th, fp32_geom=True, out=out, timing=True)
    tm = r.timing()
    st = r.stats()
    rays = P * V * H * W
    per_launch = algorithmic_bytes(st, cfg.C, 2, W, with_tfinal=False) / max(tm["n_render"], 1)
    avg = tm["render"] / max(tm["n_render"], 1) / 1e3
    del F, A, out
    return {"workload": f"precision form: BF16 storage, FP32 geometry, {P} poses x {V} cameras at {H}x{W} ({rays} rays)",
            "mrays_s": round(rays / t / 1e6, 2), "ms_per_step": round(t * 1e3, 3),
            "render_ms": round(tm["render"], 3),
            "render_hbm_frac": round(per_launch / avg / 1e9 / HBM_PEAK_GBS, 4),
            "render_launches": tm["n_render"], "avg_launch_us": round(avg * 1e6, 2),
            "samples": st["samples"], "tile_rays": st["tile_rays"], "written_rays": written_rays(st, W),
            "algorithmic_bytes_per_launch": int(per_launch),
            "algorithmic_bytes_per_sample": 2 * (cfg.C + 1) + 4}


def depth_leg(args, r, sig, feat, out, fp32_geom, torch, C, es, rays):
    """Depth buffer of hybrid rendering on the main workload: the forward maps
    plus, per ray, the distance to the first composited sample with density
    above the median leaf density; timed against the plain forward."""
    F, A, T = out
    D = torch.empty_like(A)
    th = float(sig.float().median())
    outd = (F, A, T, D)
    t_plain = _timed(torch, lambda: r.render(sig, feat, args.lambda_th, fp32_geom=fp32_geom, out=out),
                     args.proposal_steps)
    t_depth = _timed(torch, lambda: r.render_depth(sig, feat, th, args.lambda_th, fp32_geom=fp32_geom, out=outd),
                     args.proposal_steps)
    r.render_depth(sig, feat, th, args.lambda_th, fp32_geom=fp32_geom, out=outd, timing=True)
    tm = r.timing()
    st = r.stats()
    per_launch = (algorithmic_bytes(st, C, es, r.W) + 4 * written_rays(st, r.W)) / max(tm["n_render"], 1)
    avg = tm["render"] / max(tm["n_render"], 1) / 1e3
    finite = int(torch.isfinite(D).sum())
    del D, outd
    return {"workload": "depth buffer on the main workload (density threshold = median leaf density)",
            "mrays_s": round(rays / t_depth / 1e6, 2), "ms_per_step": round(t_depth * 1e3, 3),
            "plain_ms_per_step": round(t_plain * 1e3, 3),
            "overhead": round(t_depth / t_plain - 1.0, 4),
            "render_ms": round(tm["render"], 3),
            "render_hbm_frac": round(per_launch / avg / 1e9 / HBM_PEAK_GBS, 4),
            "rays_with_depth": finite}


def sh_leg(args, r, scene, out, fp32_geom, torch, C, rays, nsh=9):
    """View-dependent features on the main workload: nsh real-SH coefficient
    blocks of C channels per leaf (seeded), canonical direction from the
    dominant bone's rotation."""
    import numpy as np
    rng = np.random.default_rng(40)
    sig = torch.from_numpy(scene.sigma).cuda()
    k = torch.from_numpy(rng.normal(size=(scene.n, nsh, C)).astype(np.float32)).cuda()
    t = _timed(torch, lambda: r.render_sh(sig, k, args.lambda_th, fp32_geom=fp32_geom, out=out), args.proposal_steps)
    r.render_sh(sig, k, args.lambda_th, fp32_geom=fp32_geom, out=out, timing=True)
    tm = r.timing()
    st = r.stats()
    # per composited sample: sigma, the nsh x C coefficients, the winner id, the dominant bone
    per_sample = 4 * (1 + nsh * C) + 4 + 1
    per_launch = (st["samples"] * per_sample + written_rays(st, r.W) * (4 * (C + 2))) / max(tm["n_render"], 1)
    avg = tm["render"] / max(tm["n_render"], 1) / 1e3
    del k
    return {"workload": f"view-dependent features on the main workload: H = {nsh} SH blocks of C = {C}, FP32",
            "mrays_s": round(rays / t / 1e6, 2), "ms_per_step": round(t * 1e3, 3),
            "render_ms": round(tm["render"], 3), "algorithmic_bytes_per_sample": per_sample,
            "render_hbm_frac": round(per_launch / avg / 1e9 / HBM_PEAK_GBS, 4)}


def shading_leg(args, r, F, torch, C, maps=32):
    """The Light shading network (FP16 matrix cores) on `maps` rendered feature
    maps of the main workload; achieved TFLOP/s of its convolutions."""
    import scenegen as sgm
    H, W = F.shape[-2], F.shape[-1]
    Fm = F.reshape(-1, C, H, W)[:maps].contiguous()
    r.set_shading_weights(C, sgm.make_shading_weights(C))
    out = torch.empty((maps, 4, H, W), dtype=torch.float32, device=F.device)
    t = _timed(torch, lambda: r.shade(Fm, out=out), args.proposal_steps)
    # multiply-adds of the 3x3 convolutions (layer 0 counted with its C input
    # channels, not the 32 it is padded to) and the head
    px = maps * H * W
    macs = 9 * px * (C * 32 + 32 * 32) + 9 * px // 4 * (32 * 64 + 64 * 64) + 9 * px // 16 * (64 * 128 + 128 * 128) \
        + 9 * px // 64 * (128 * 256 + 256 * 256) + 9 * px // 16 * (384 * 128 + 128 * 128) \
        + 9 * px // 4 * (192 * 64 + 64 * 64) + 9 * px * (96 * 32 + 32 * 32) + px * 32 * 4
    tflops = 2 * macs / t / 1e12
    bound = shading_layer_bound(maps, H, W, C)
    return {"workload": f"Light shading network, {maps} maps of {H}x{W}, C = {C}, FP16 operands, FP32 accumulation",
            "ms": round(t * 1e3, 3), "maps_per_s": round(maps / t, 1), "tflop_per_map": round(2 * macs / maps / 1e12, 4),
            "achieved_tflops": round(tflops, 1), "peak_tflops": 2500.0, "frac": round(tflops / 2500.0, 4),
            "layer_bound_ms": round(bound * 1e3, 3), "frac_of_layer_bound": round(bound / t, 4)}


def shading_layer_bound(maps, H, W, C, peak_flops=2.5e15, peak_bytes=8e12):
    """Lower bound of the shading network's time: per layer the larger of its
    FP16 matrix-core time (2 x 9 x Cin x Cout per output pixel at 2.5 PFLOP/s)
    and its HBM time (each input read once - a decoder's deeper input at half
    resolution - and the output written once, FP16 NHWC, at 8 TB/s), plus the
    input conversion (16 FP32 planes in, 32 FP16 channels out) and the three
    2x2 max pools, which are HBM-bound.  The 1x1 head runs in the last
    convolution, whose output is its 4 FP32 channels."""
    px = maps * H * W
    # (resolution divisor, C1 same-resolution inputs, C2 half-resolution inputs, Cout, real Cin for the flops)
    convs = [(1, 32, 0, 32, C), (1, 32, 0, 32, 32), (2, 32, 0, 64, 32), (2, 64, 0, 64, 64), (4, 64, 0, 128, 64),
             (4, 128, 0, 128, 128), (8, 128, 0, 256, 128), (8, 256, 0, 256, 256), (4, 128, 256, 128, 384),
             (4, 128, 0, 128, 128), (2, 64, 128, 64, 192), (2, 64, 0, 64, 64), (1, 32, 64, 32, 96),
             (1, 32, 0, 32, 32)]
    t = 0.0
    for i, (div, c1, c2, co, cin) in enumerate(convs):
        n = px // (div * div)
        flops = 2 * 9 * cin * co * n
        out_bytes = 4 * 4 * n if i == len(convs) - 1 else 2 * n * co   # the last one writes the head's output
        bytes_ = 2 * n * c1 + out_bytes + 2 * (n // 4) * c2 + 2 * 9 * (c1 + c2) * co
        t += max(flops / peak_flops, bytes_ / peak_bytes)
    t += px * (4 * C + 2 * 32) / peak_bytes                                          # conversion
    t += sum((px // (d * d)) * 2 * c * 5 / 4 for d, c in ((1, 32), (2, 64), (4, 128))) / peak_bytes  # pools
    return t


def adjoint_leg(args, art, sg, torch):
    """Differentiation form: L = 1/2 |F - F*|^2 over 4 cameras at 512^2, one
    pose; the adjoint kernel re-traverses every ray (per-ray recomputation)."""
    cfg = sg.CONFIGS["grad"]
    scene = sg.make_scene(cfg)
    P, V, H, W = cfg.n_poses, cfg.n_views, cfg.height, cfg.width
    r = art.Renderer(0)
    r.set_scene(scene)
    r.set_poses(*sg.make_poses(scene.J, P, cfg.pose_seed0))
    r.set_cameras(*sg.make_cameras(scene, V, H, W), H, W)
    sig = torch.from_numpy(scene.sigma).cuda()
    feat = torch.from_numpy(scene.feat).cuda()
    tgt = torch.from_numpy(sg.make_targets(P, V, cfg.C, H, W, cfg.target_seed)).cuda()
    F, A, T = r.render(sig, feat, args.lambda_th)
    st = r.stats()
    dF = (F - tgt).contiguous()
    ds = torch.zeros_like(sig)
    df = torch.zeros_like(feat)
    t = _timed(torch, lambda: r.backward(sig, feat, F, T, dF, d_sigma=ds, d_feat=df), args.proposal_steps)
    r.backward(sig, feat, F, T, dF, d_sigma=ds, d_feat=df, timing=True)
    tm = r.timing()
    # as the autograd backward runs it: the forward's posed octrees reused
    r.render(sig, feat, args.lambda_th, out=(F, A, T))
    t_reuse = _timed(torch, lambda: r.backward(sig, feat, F, T, dF, d_sigma=ds, d_feat=df, reuse_build=True),
                     args.proposal_steps)
    rays = P * V * H * W
    # per composited sample: the re-gathered density, features and leaf index
    # (72 B) and the gradient atomics (C + 1 floats); per ray of a non-empty
    # tile: dL/dF, F and T_final
    per_sample = 4 * (cfg.C + 1) + 4 + 4 * (cfg.C + 1)
    per_ray = 4 * cfg.C + 4 * cfg.C + 4
    alg = st["samples"] * per_sample + st["tile_rays"] * per_ray
    kern_ms = tm["render"] / max(tm["n_render"], 1)
    # the segmented adjoint: the forward records a checkpoint every `every`
    # samples of a ray (K per ray), the adjoint runs the K + 1 segments of
    # every ray in parallel; the records it reads (C + 4 words each) count
    # in its algorithmic bytes
    r.render(sig, feat, args.lambda_th, out=(F, A, T), timing=True)
    fwd_ms = r.timing()["render"]
    seg = []
    for K, every in ((4, 48), (6, 36), (8, 32)):
        Fc, Ac, Tc, ck = r.render_ckpt(sig, feat, args.lambda_th, K=K, every=every, timing=True)
        fwd_ck_ms = r.timing()["render"]
        r.backward(sig, feat, Fc, Tc, dF, d_sigma=ds, d_feat=df, reuse_build=True, ckpt=ck)   # warm-up
        t_seg = _timed(torch, lambda: r.backward(sig, feat, Fc, Tc, dF, d_sigma=ds, d_feat=df, reuse_build=True,
                                                 ckpt=ck), args.proposal_steps)
        r.backward(sig, feat, Fc, Tc, dF, d_sigma=ds, d_feat=df, reuse_build=True, ckpt=ck, timing=True)
        tms = r.timing()
        k_ms = tms["render"] / max(tms["n_render"], 1)
        recs = int(ck[1].sum())
        alg_s = alg + recs * 4 * (cfg.C + 4)
        seg.append({"K": K, "every": every, "records": recs, "adjoint_kernel_ms": round(k_ms, 4),
                    "ms_per_call_reusing_forward_octrees": round(t_seg * 1e3, 3),
                    "adjoint_hbm_frac": round(alg_s / (k_ms * 1e-3) / 8e12, 4),
                    "forward_kernel_ms_with_checkpoints": round(fwd_ck_ms, 4)})
        del Fc, Ac, Tc, ck
    best = min(seg, key=lambda x: x["adjoint_kernel_ms"])
    return {"workload": f"adjoint: {P} pose x {V} cameras at {H}x{W} ({rays} rays), L2 loss to seeded targets",
            "mrays_s": round(rays / t / 1e6, 2), "ms_per_call": round(t * 1e3, 3),
            "ms_per_call_reusing_forward_octrees": round(t_reuse * 1e3, 3),
            "adjoint_kernel_ms": round(kern_ms, 4), "samples": st["samples"], "tile_rays": st["tile_rays"],
            "algorithmic_bytes_per_launch": int(alg),
            "algorithmic_bytes_per_sample": per_sample, "algorithmic_bytes_per_ray": per_ray,
            "adjoint_hbm_frac": round(alg / (kern_ms * 1e-3) / 8e12, 4),
            "forward_kernel_ms": round(fwd_ms, 4),
            "segmented": {"best": best, "sweep": seg,
                          "note": "art_render_ckpt + art_backward_ckpt: K + 1 segments per ray from the "
                                  "forward's records; algorithmic bytes add the records read"}}


def adjoint_main_leg(args, r, sig, feat, out, torch, C, rays):
    """The adjoint kernel on the main workload (30 poses x 8 cameras at
    512^2): L = 1/2 |F - F*|^2 to seeded N(0, 1) targets, one backward call
    after the forward.  The differentiation workload (1 pose x 4 cameras)
    holds about 2,600 non-empty tiles, fewer than the GPU has wave slots, so
    its time is the serial chain of its longest rays; here the kernel has
    enough tiles to show its throughput."""
    F, A, T = out
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    dF = torch.randn(F.shape, generator=g, device="cuda", dtype=torch.float32)
    dF.sub_(F).neg_()                                     # dL/dF = F - F*
    ds = torch.zeros_like(sig)
    df = torch.zeros_like(feat)
    r.render(sig, feat, args.lambda_th, out=out)
    st = r.stats()
    r.backward(sig, feat, F, T, dF, None, args.lambda_th, d_sigma=ds, d_feat=df, reuse_build=True)   # warm-up
    r.render(sig, feat, args.lambda_th, out=out)
    r.backward(sig, feat, F, T, dF, None, args.lambda_th, d_sigma=ds, d_feat=df, reuse_build=True, timing=True)
    tm = r.timing()
    per_sample = 4 * (C + 1) + 4 + 4 * (C + 1)
    per_ray = 4 * C + 4 * C + 4
    alg = st["samples"] * per_sample + st["tile_rays"] * per_ray
    kern_ms = tm["render"] / max(tm["n_render"], 1)
    del dF, ds, df
    return {"workload": "adjoint on the main workload (30 poses x 8 cameras at 512x512), L2 loss to seeded targets",
            "adjoint_kernel_ms": round(kern_ms, 3), "launches": tm["n_render"], "samples": st["samples"],
            "algorithmic_bytes_per_launch": int(alg / max(tm["n_render"], 1)),
            "adjoint_hbm_frac": round(alg / max(tm["n_render"], 1) / (kern_ms * 1e-3) / 8e12, 4),
            "mrays_s_kernel": round(rays / (tm["render"] * 1e-3) / 1e6, 2)}


def adjoint_main_only_leg(args, art, sg, torch):
    """The adjoint on the main workload on its own (for counter runs): the
    forward, then adjoint_main_leg."""
    cfg = sg.CONFIGS["full"]
    scene = sg.make_scene(cfg)
    P, V, H, W = cfg.n_poses, cfg.n_views, cfg.height, cfg.width
    r = art.Renderer(0)
    r.set_scene(scene)
    r.set_poses(*sg.make_poses(scene.J, P, cfg.pose_seed0))
    r.set_cameras(*sg.make_cameras(scene, V, H, W), H, W)
    sig = torch.from_numpy(scene.sigma).cuda()
    feat = torch.from_numpy(scene.feat).cuda()
    F = torch.empty((P, V, cfg.C, H, W), dtype=torch.float32, device="cuda")
    A = torch.empty((P, V, H, W), dtype=torch.float32, device="cuda")
    T = torch.empty_like(A)
    return adjoint_main_leg(args, r, sig, feat, (F, A, T), torch, cfg.C, P * V * H * W)


def train_leg(args, art, sg, torch):
    """FLUT training step on the differentiation workload (1 pose x 4 cameras at
    512^2, C = 16, FP32): render, L2 map loss to seeded targets, adjoint,
    voxel regularisation term (lambda_vrt = 0.05), Adam on sigma and features."""
    cfg = sg.CONFIGS["grad"]
    scene = sg.make_scene(cfg)
    P, V, H, W = cfg.n_poses, cfg.n_views, cfg.height, cfg.width
    r = art.Renderer(0)
    r.set_scene(scene)
    r.set_poses(*sg.make_poses(scene.J, P, cfg.pose_seed0))
    r.set_cameras(*sg.make_cameras(scene, V, H, W), H, W)
    sig = torch.from_numpy(scene.sigma).cuda()
    feat = torch.from_numpy(scene.feat).cuda()
    tgt = torch.from_numpy(sg.make_targets(P, V, cfg.C, H, W, cfg.target_seed)).cuda()
    st = r.train_state(sig, feat)
    losses = []
    t = _timed(torch, lambda: losses.append(r.train_step(sig, feat, st, tgt, lr=1e-2, lambda_vrt=0.05)),
               args.proposal_steps)
    t_vrt = _timed(torch, lambda: r.vrt(feat, 0.05), args.proposal_steps)
    rays = P * V * H * W
    return {"workload": f"FLUT training step: {P} pose x {V} cameras at {H}x{W} ({rays} rays), L2 map loss, "
                        f"VRT lambda 0.05, Adam lr 1e-2",
            "ms_per_step": round(t * 1e3, 3), "mrays_s": round(rays / t / 1e6, 2),
            "vrt_ms": round(t_vrt * 1e3, 3),
            "loss_first": round(losses[0]["total"], 6), "loss_last": round(losses[-1]["total"], 6)}


def proposal_leg(args, art, sg, torch):
    """Learned ray-interval proposal vs the plain renderer on the proposal
    workload (60 poses x 16 cameras at 1024^2, C = 16, FP32): the network is
    trained on the GPU (own kernels) on labels of the plain renderer, then both
    renderers are timed over the whole batch; the proposal's error against the
    plain maps is measured on the first poses, together with the untrained
    network (the control)."""
    cfg = sg.CONFIGS["proposal"]
    scene = sg.make_scene(cfg)
    P, V, H, W = cfg.n_poses, cfg.n_views, cfg.height, cfg.width
    poses = sg.make_poses(scene.J, P, cfg.pose_seed0)
    K, c2w = sg.make_cameras(scene, V, H, W)
    r = art.Renderer(0)
    r.set_scene(scene)
    r.set_poses(*poses)
    r.set_cameras(K, c2w, H, W)
    sig = torch.from_numpy(scene.sigma).cuda()
    feat = torch.from_numpy(scene.feat).cuda()
    lam = args.lambda_th
    t0 = time.perf_counter()
    lab = r.proposal_labels(sig, feat, lam)
    hit = (lab[..., 0] <= lab[..., 1]).cpu().numpy()
    ids = sg.sample_training_rays(args.train_rays, P, V, H, W, hit_mask=hit, seed=cfg.ray_seed)
    del hit
    od, pose, tgt = r.proposal_gather(torch.from_numpy(ids).cuda(), lab)
    del lab
    n_train = int(0.9 * len(ids))
    theta0 = sg.make_mlp_init(scene.J, seed=cfg.mlp_seed)
    r.set_proposal_weights(theta0)
    r.set_proposal_loss(args.proposal_loss, (args.tau_near, args.tau_far))
    val0, _ = r.proposal_grad(od[n_train:n_train + 65536], pose[n_train:n_train + 65536], tgt[n_train:n_train + 65536])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    losses = r.proposal_train(od[:n_train], pose[:n_train], tgt[:n_train], batch=16384, steps=args.train_steps,
                              lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    val1, _ = r.proposal_grad(od[n_train:n_train + 65536], pose[n_train:n_train + 65536], tgt[n_train:n_train + 65536])
    margin = args.margin_h or r.calibrate_proposal_margin(od[n_train:], pose[n_train:], tgt[n_train:],
                                                          quantile=args.margin_quantile)
    print(f"[bench] proposal trained: {args.train_steps} steps in {t_train:.2f} s, validation loss "
          f"{val0:.4f} -> {val1:.4f}; start margin {margin:.1f} h", file=sys.stderr, flush=True)
    theta1 = r.get_proposal_weights()
    # the untrained control's own calibrated margin (same rule, same held-out rays)
    r.set_proposal_weights(theta0)
    mu = args.margin_h or r.calibrate_proposal_margin(od[n_train:], pose[n_train:], tgt[n_train:],
                                                      quantile=args.margin_quantile)
    r.set_proposal_weights(theta1)
    del od, pose, tgt
    F = torch.empty((P, V, cfg.C, H, W), dtype=torch.float32, device="cuda")
    A = torch.empty((P, V, H, W), dtype=torch.float32, device="cuda")
    out = (F, A, None)
    rays = P * V * H * W
    t_plain = _timed(torch, lambda: r.render(sig, feat, lam, out=out), args.proposal_steps)
    st_plain = r.stats()
    kw = dict(margin_h=margin, f2_tau=args.f2_tau, near_only=True)
    t_prop = _timed(torch, lambda: r.render_proposal(sig, feat, None, lam, out=out, **kw), args.proposal_steps)
    st = r.stats()
    r.render_proposal(sig, feat, None, lam, out=out, timing=True, **kw)
    tm = r.timing()
    del F, A, out
    # error on the first poses (plain vs trained vs untrained network)
    Pe = min(args.err_poses, P)
    r.set_poses(poses[0][:Pe], poses[1][:Pe], poses[2][:Pe])
    F0, _, _ = r.render(sig, feat, lam, want_tfinal=False)
    st0 = r.stats()
    F1, _, _ = r.render_proposal(sig, feat, None, lam, want_tfinal=False, **kw)
    st1 = r.stats()
    den = float(F0.abs().sum())
    err_mean = float((F1 - F0).abs().sum()) / den
    err_max = max(float((F1[p, v] - F0[p, v]).abs().max() / F0[p, v].abs().max())
                  for p in range(Pe) for v in range(V))
    r.set_proposal_weights(theta0)
    Fu, _, _ = r.render_proposal(sig, feat, None, lam, want_tfinal=False, **dict(kw, margin_h=mu))
    stu = r.stats()
    err_u = float((Fu - F0).abs().sum()) / den
    r.set_proposal_weights(theta1)
    del F0, F1, Fu
    return {
        "workload": (f"learned proposal: depth {cfg.depth} octree, {scene.n} leaves, {scene.J} bones, C={cfg.C}, "
                     f"{P} poses x {V} cameras at {H}x{W} ({rays} rays), lambda_th={lam}"),
        "plain_mrays_s": round(rays / t_plain / 1e6, 2),
        "proposal_mrays_s": round(rays / t_prop / 1e6, 2),
        "speedup": round(t_plain / t_prop, 4),
        "rel_mean_err": err_mean,
        "rel_max_err": err_max,
        "err_poses": Pe,
        "margin_h": round(margin, 2),
        "margin_rule": (f"calibrated: {100 * args.margin_quantile:g}% quantile of late starts on held-out rays"
                        if not args.margin_h else "fixed"),
        "loss": (args.proposal_loss if args.proposal_loss == "smooth_l1" else
                 f"pinball on rays with a sample (tau_near {args.tau_near}, tau_far {args.tau_far}), "
                 f"SmoothL1 on empty labels"),
        "interval": "near end only (traversal from t_a + u_near (t_b - t_a) - m to t_b)",
        "f2_tau": args.f2_tau,
        "partition_steps_plain": st_plain["steps"],
        "partition_steps_proposal": st["steps"],
        "rounds_plain": st_plain["rounds"],
        "rounds_proposal": st["rounds"],
        "proposal_rays": st["proposal_rays"],
        "fallback_rate": round(st["fallbacks"] / max(st["proposal_rays"], 1), 4),
        "inference_ms": round(tm["proposal"], 3),
        "render_ms": round(tm["render"], 3),
        "untrained_control": {"rel_mean_err": err_u, "margin_h": round(mu, 2),
                              "partition_steps_first_poses": stu["steps"],
                              "partition_steps_plain_first_poses": st0["steps"],
                              "fallback_rate": round(stu["fallbacks"] / max(stu["proposal_rays"], 1), 4)},
        "trained_first_poses": {"partition_steps": st1["steps"], "rounds": st1["rounds"],
                                "plain_rounds": st0["rounds"]},
        "training": {"rays": int(len(ids)), "train_rays": n_train, "steps": args.train_steps, "batch": 16384,
                     "seconds": round(t_train, 3), "first_loss": float(losses[0]), "last_loss": float(losses[-1]),
                     "val_loss_before": val0, "val_loss_after": val1,
                     "setup_seconds": round(time.perf_counter() - t0, 2)},
    }


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the renderer has no multi-GPU path "
              "(each GPU would render its own poses/views with no exchange); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2202_05628_amd as art
    import scenegen as sg

    if args.leg:
        legs = {"bf16": bf16_leg, "adjoint": adjoint_leg, "adjoint_main": adjoint_main_only_leg, "train": train_leg,
                "proposal": proposal_leg}
        print(json.dumps({args.leg: legs[args.leg](args, art, sg, torch)}), flush=True)
        return

    cfg = sg.CONFIGS[args.config]
    scene = sg.make_scene(cfg)
    P = args.poses or cfg.n_poses
    poses = sg.make_poses(scene.J, P, cfg.pose_seed0)
    K, c2w = sg.make_cameras(scene, cfg.n_views, cfg.height, cfg.width)
    r = art.Renderer(0)
    r.set_scene(scene)
    r.set_poses(*poses)
    r.set_cameras(K, c2w, cfg.height, cfg.width)
    dt = torch.bfloat16 if cfg.storage == "bf16" else torch.float32
    sig = torch.from_numpy(scene.sigma).cuda().to(dt).contiguous()
    feat = torch.from_numpy(scene.feat).cuda().to(dt).contiguous()
    Fm = torch.empty((P, cfg.n_views, cfg.C, cfg.height, cfg.width), dtype=torch.float32, device="cuda")
    Am = torch.empty((P, cfg.n_views, cfg.height, cfg.width), dtype=torch.float32, device="cuda")
    Tm = torch.empty_like(Am)
    out = (Fm, Am, Tm)
    fp32_geom = cfg.storage == "bf16"

    copy_gbs = copy_probe(torch) if args.copy_probe else None
    for i in range(args.warmup):
        r.render(sig, feat, args.lambda_th, fp32_geom=fp32_geom, out=out)
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    render_ms = 0.0
    n_render = 0
    stages = {"fk": 0.0, "skin": 0.0, "build": 0.0, "bin": 0.0, "render": 0.0}
    t0 = time.perf_counter()
    for i in range(args.steps):
        r.render(sig, feat, args.lambda_th, fp32_geom=fp32_geom, timing=True, out=out)
        tm = r.timing()
        render_ms += tm["render"]
        n_render += tm["n_render"]
        for k in stages:
            stages[k] += tm[k]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = r.stats()
    rays_per_step = P * cfg.n_views * cfg.height * cfg.width
    value = rays_per_step * args.steps / elapsed / 1e6
    es = 2 if cfg.storage == "bf16" else 4
    bytes_call = algorithmic_bytes(st, cfg.C, es, cfg.width)
    launches_per_call = n_render / args.steps
    per_launch_bytes = bytes_call / launches_per_call
    avg_launch_s = render_ms / n_render / 1e3
    achieved = per_launch_bytes / avg_launch_s / 1e9
    hit = st["hit_rays"] / max(st["rays"], 1)
    workload = (f"plain renderer {cfg.name}: depth {cfg.depth} octree, {scene.n} leaves, "
                f"{scene.J} bones, C={cfg.C}, {P} poses x {cfg.n_views} cameras at "
                f"{cfg.height}x{cfg.width}, lambda_th={args.lambda_th}")
    line = {
        "metric": "feature-map Mrays/s (C=16) learned-proposal vs plain at <=1e-3 rel err; %HBM peak",
        "value": round(value, 2),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-storage/f32" if cfg.storage == "bf16" else "f32",
        "data": "synthetic (seeded animal-shaped octree, ring cameras, random poses)",
        "config": {
            "workload": workload,
            "poses": P, "views": cfg.n_views, "height": cfg.height, "width": cfg.width,
            "C": cfg.C, "leaves": scene.n, "depth": cfg.depth, "storage": cfg.storage,
            "geometry": "fp32" if fp32_geom else "fp64",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(workload),
            "kernel": "k_render (forward compositing)",
            "render_source_hash": render_source_hash(),
            "copy_probe_GBps": None if copy_gbs is None else round(copy_gbs, 1),
            "launches_per_step": launches_per_call,
            "avg_launch_us": round(avg_launch_s * 1e6, 2),
            "algorithmic_bytes_per_launch": int(per_launch_bytes),
        },
        "stages_ms_per_step": {k: round(v / args.steps, 3) for k, v in stages.items()},
        "hit_fraction": round(hit, 4),
        "samples_per_hit_ray": round(st["samples"] / max(st["hit_rays"], 1), 2),
        "collisions_per_pose": st["collisions"] // P,
        "bricks_per_pose": st["bricks"] // P,
        "tile_list_entries_per_pose": st["list_entries"] // P,
        "traversal_rounds_per_pose": st["rounds"] // P,
        "partition_steps_per_pose": st["steps"] // P,
        "launches_per_step": st["launches"],
    }
    if not args.no_forms:
        print("[bench] depth buffer", file=sys.stderr, flush=True)
        line["depth_form"] = depth_leg(args, r, sig, feat, out, fp32_geom, torch, cfg.C, es, rays_per_step)
        print("[bench] shading network", file=sys.stderr, flush=True)
        line["shading_form"] = shading_leg(args, r, Fm, torch, cfg.C)
        if cfg.storage == "f32":
            print("[bench] view-dependent features", file=sys.stderr, flush=True)
            line["sh_form"] = sh_leg(args, r, scene, out, fp32_geom, torch, cfg.C, rays_per_step)
            print("[bench] adjoint on the main workload", file=sys.stderr, flush=True)
            line["adjoint_main_workload"] = adjoint_main_leg(args, r, sig, feat, out, torch, cfg.C, rays_per_step)
    del Fm, Am, Tm, out
    torch.cuda.empty_cache()
    if not args.no_forms:
        print("[bench] BF16 precision form and adjoint", file=sys.stderr, flush=True)
        line["bf16_form"] = bf16_leg(args, art, sg, torch)
        torch.cuda.empty_cache()
        line["adjoint_form"] = adjoint_leg(args, art, sg, torch)
        torch.cuda.empty_cache()
        line["train_step"] = train_leg(args, art, sg, torch)
        torch.cuda.empty_cache()
    if not args.no_proposal:
        print("[bench] learned proposal vs plain (proposal workload)", file=sys.stderr, flush=True)
        line["proposal"] = proposal_leg(args, art, sg, torch)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(scene, poses, K, c2w, cfg.height, cfg.width,
                                            args.lambda_th, args.cpu_seconds)
        line["cpu_baseline"]["other_workloads"] = cpu_other_configs(sg, scene, args.lambda_th)
        if not args.no_forms:
            print("[bench] errors of the extra forms against the FP64 oracle", file=sys.stderr, flush=True)
            errs = oracle_checks(art, sg, torch, args.lambda_th)
            line["bf16_form"]["error_vs_fp64_oracle"] = errs["bf16_form"]
            line["adjoint_form"]["gradient_vs_fp64_oracle"] = errs["adjoint_form"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
