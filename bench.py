"""Throughput benchmark: KF propagate+update steps per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the uneven-multiplicity batch (64 events, track counts ~ Poisson
with mean ~ U(200, 4000), 60 noise hits per track, ten barrel layers plus
2 x 7 disks, |eta| < 2.5, 0.02 X0 per layer), synthetic.  One timed step is
one pass of the whole finding path over the batch, inputs resident in HBM:
seed every track from its first three hits (kf_seed), Kalman-fit the three
seed hits (kf_fit), then kf_find (hit binning, seed ordering, the persistent
finding kernel), replayed as one captured HIP graph (kf_find_batched) after
the autotuner has picked the finding width and tile order.  A KF step is one
propagation of a track or candidate to a surface together with its
update(s): the three seed-fit steps per seed plus the finding kernel's
propagations (counted by the kernel itself).

Prints ONE JSON line: metric, value, the HBM roofline of the dominant kernel
(the finding kernel: algorithmic bytes of the per-layer state-through-memory
model, 250 B per propagation plus 108 B per extra child kept, times its
event counters, over its HIP-event time; its arithmetic rate beside), the
FP64 oracle timed on the host cores (all of them and one thread), the
finding pass over 512 events (a working set far above the 256 MB Infinity
Cache), and the fit kernels' figures (the per-layer step against 244 B).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3       # MI355X vector FP32 (packed)
VECTOR_PEAK_TFLOPS = 78.6      # MI355X vector FP64, and FP32 without packed math (unpacked)

# Algorithmic bytes of one per-layer fit step (the state crosses HBM between
# layers, FP32 storage): state 24 + covariance 84 read and written, hit
# x, y, z, su, sv 20, chi2 read and written 8.
FIT_BYTES_PER_STEP = 2 * (24 + 84) + 20 + 8
# What the per-layer kernel actually moves per step besides: the hit index
# and layer index (4 + 4) and ndf and status read and written (16).
PER_LAYER_BYTES_PER_STEP = FIT_BYTES_PER_STEP + 8 + 16
# Algorithmic bytes of one finding step, the same per-layer model: the
# parent's state and covariance read (108), hit index, hit count and chi2
# (12), the layer's hits amortised over its candidates (~24 at the finding
# workloads' occupancy) and one child written (108): ~250 B, plus 108 B for
# every further child kept.
FIND_BYTES_PER_STEP = 250.0
FIND_BYTES_PER_EXTRA_CHILD = 108.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--width", type=int, default=0,
                    help="finding workgroup width; 0 = autotune width and tile order")
    ap.add_argument("--largest-first", action="store_true",
                    help="with --width: events largest first in the tile order")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fit", action="store_true")
    ap.add_argument("--no-clean", action="store_true")
    ap.add_argument("--no-material", action="store_true")
    ap.add_argument("--no-field-find", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--fit-tracks", type=int, default=4_000_000)
    ap.add_argument("--field-tracks", type=int, default=1_000_000)
    return ap.parse_args()


# HBM bytes per launch from the committed rocprofv3 counter summary, used
# only while the finding kernel's sources are the ones it was measured on
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "find_pass_batch64_hbm_counters.json")
KERNEL_SOURCES = ["kf_find.hip", "kf_find.hpp", "kf_math.hpp", "kf_mlp.hpp", "kf_internal.hpp",
                  "kf_matmap.hpp", "kf_steer.hpp"]
FIND_KERNEL = "kfmi::find_kernel<float, double, double, false, false, false, false>"


FIT_SOURCES = ["kf_fit.hip", "kf_math.hpp", "kf_mlp.hpp", "kf_internal.hpp", "kf_matmap.hpp"]
PER_LAYER_KERNEL = "kfmi::fit_kernel<float, double, double, false, false, false> (per layer)"


def measured_traffic(kernel, sources=KERNEL_SOURCES, hash_key="kernel_source_hash"):
    """HBM bytes per dispatch of `kernel` from the committed counter summary,
    or None when the kernel's sources changed since it was taken."""
    import hashlib
    try:
        with open(TRAFFIC_JSON) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    for s in sources:
        with open(os.path.join(ROOT, "paper_1906_02253_amd", "csrc", s), "rb") as f:
            h.update(f.read())
    if d.get(hash_key) != h.hexdigest()[:16]:
        return None
    k = d.get("kernels", {}).get(kernel)
    return k["hbm_bytes"] if k else None


def find_roofline(cnt, kernel_ms, oc, traffic=None, kernel=None):
    """HBM roofline of the finding kernel from its event counters
    (propagations cnt[0], children kept cnt[7]) and its mean kernel time;
    its arithmetic rate beside."""
    props, kept = float(cnt[0]), float(cnt[7])
    nbytes = FIND_BYTES_PER_STEP * props + FIND_BYTES_PER_EXTRA_CHILD * (kept - props)
    gbs = nbytes / (kernel_ms * 1e-3) / 1e9
    flops = find_flops(cnt, oc)
    tf = flops / (kernel_ms * 1e-3) / 1e12
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
            "kernel_ms": kernel_ms, "bytes_per_launch": nbytes,
            "bytes_model": "250 B per propagation + 108 B per child kept beyond one",
            "children_per_propagation": kept / max(props, 1.0),
            "alu": {"achieved_tflops": tf, "peak_fp32_packed_tflops": FP32_PEAK_TFLOPS,
                    "frac": tf / FP32_PEAK_TFLOPS,
                    "peak_unpacked_tflops": VECTOR_PEAK_TFLOPS,
                    "frac_unpacked": tf / VECTOR_PEAK_TFLOPS, "flops_per_launch": flops},
            "events_per_launch": cnt.tolist()}


def find_flops(cnt, oc):
    """Algorithmic flops of the finding kernel from its event counters and the
    operation counts of its arithmetic (special-function calls counted as one)."""
    props, upd, chi2, newton, disk = [float(c) for c in cnt[:5]]
    f = lambda k: oc[k]["ops"] + oc[k]["sfu"]
    per_prop = f("nav_fixed") + f("barrel_setup") + f("transport_barrel") + f("window")
    return (props * per_prop + newton * f("newton_eval") + disk * f("disk_eval")
            + chi2 * f("hit_test") + upd * f("update"))


def build_fit_set(n_total, n_unique=1_000_000, chunk=250_000, seed=3):
    """Fit sample of the precision workload's distribution (pT 0.3 / 100 GeV,
    hit sigma_u log-uniform 0.002-0.01 cm, sigma_v = 5 sigma_u, ten barrel
    layers, no material): n_unique generated tracks replicated at distinct
    addresses up to n_total, hits step-major (step k of track i is hit k*ld+i)."""
    import eventgen as E
    ld = (n_total + 63) // 64 * 64
    ms = 10
    m = min(n_unique, n_total)
    bx = np.zeros((ms, m), np.float32)
    by, bz_ = np.zeros_like(bx), np.zeros_like(bx)
    bsu, bsv = np.full_like(bx, 0.01), np.full_like(bx, 0.05)
    bl = np.zeros((ms, m), np.int32)
    blseq = np.full((ms, m), -1, np.int32)
    done, k = 0, 0
    geom = E.geometry.barrel10(x0=0.0)
    while done < m:
        n = min(chunk, m - done)
        rng = np.random.default_rng(seed * 1000 + k)
        ev = E.make_event(rng, geom, n, E.pt_two_values(0.3, 100.0), 1.0,
                          sig_fn=E.sig_loguniform(0.002, 0.01, 5.0))
        cols = np.arange(done, done + n)
        for s in range(ms):
            hi = ev.seq_hit[:, s]
            msk = hi >= 0
            src = hi[msk]
            c = cols[msk]
            bx[s, c], by[s, c], bz_[s, c] = ev.x[src], ev.y[src], ev.z[src]
            bsu[s, c], bsv[s, c], bl[s, c] = ev.su[src], ev.sv[src], ev.layer[src]
            blseq[s, c] = ev.seq_layer[msk, s]
        done += n
        k += 1
    reps = (n_total + m - 1) // m

    def tile(a, fill):
        out = np.full((ms, ld), fill, a.dtype)
        out[:, :n_total] = np.tile(a, (1, reps))[:, :n_total]
        return out
    lseq = tile(blseq, -1)
    hits = dict(x=tile(bx, 0).reshape(-1), y=tile(by, 0).reshape(-1), z=tile(bz_, 0).reshape(-1),
                su=tile(bsu, 0.01).reshape(-1), sv=tile(bsv, 0.05).reshape(-1),
                layer=tile(bl, 0).reshape(-1))
    hidx = np.where(lseq >= 0, (np.arange(ms)[:, None] * ld + np.arange(ld)[None, :]), -1)
    return geom, ld, hits, lseq, hidx.astype(np.int32)


def run_fit(K, torch, n, w=None, reps=5):
    """Fused fit (plain and, given weights w, learned start) and per-layer fit
    of n tracks: kernel ms (HIP events) and rates."""
    geom, ld, hits_np, lseq_np, hidx_np = build_fit_set(n)
    hits = K.Hits(hits_np["x"], hits_np["y"], hits_np["z"], hits_np["su"], hits_np["sv"],
                  hits_np["layer"])
    lseq = torch.as_tensor(lseq_np, device="cuda")
    hidx = torch.as_tensor(hidx_np, device="cuda")
    seed_hits = hidx[:3].contiguous()
    ctx = K.Context(geom)
    tm = K.Tracks(n, ld)
    t32 = K.Tracks(n, ld, K.PREC_FP32)
    n_steps = int((lseq_np[:, :n] >= 0).sum())
    stream = torch.cuda.current_stream()
    out = {}
    legs = [("fused", 0), ("per_layer", K.PER_LAYER), ("per_layer_fp32", K.PER_LAYER | K.PREC_FP32)]
    if w is not None:
        ctx.mlp_load(w)
        legs.append(("fused_learned", K.INIT_MLP))
    for name, flags in legs:
        t = t32 if flags & K.PREC_FP32 else tm
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for r in range(-1, reps):
            ctx.seed(hits, seed_hits, t, flags & 3)
            if r >= 0:
                ev[r][0].record(stream)
            ctx.fit(t, hits, lseq, hidx, 10, flags=flags)
            if r >= 0:
                ev[r][1].record(stream)
        torch.cuda.synchronize()
        out[name] = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    gbs = n_steps * FIT_BYTES_PER_STEP / (out["per_layer"] * 1e-3) / 1e9
    gbs32 = n_steps * FIT_BYTES_PER_STEP / (out["per_layer_fp32"] * 1e-3) / 1e9
    return {"workload": f"fit of {n} tracks, precision-workload mix, 10 barrel layers, mixed "
                        f"precision (FP32 storage)",
            "kf_steps": n_steps,
            "fused_kernel_ms": out["fused"], "fused_steps_per_s": n_steps / (out["fused"] * 1e-3),
            "fused_learned_kernel_ms": out.get("fused_learned"),
            "fused_learned_steps_per_s": n_steps / (out["fused_learned"] * 1e-3)
            if "fused_learned" in out else None,
            "per_layer_ms": out["per_layer"],
            "per_layer_steps_per_s": n_steps / (out["per_layer"] * 1e-3),
            "per_layer_hbm": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": gbs / HBM_PEAK_GBS,
                              "bytes_per_step": FIT_BYTES_PER_STEP,
                              "bytes_moved_per_step": PER_LAYER_BYTES_PER_STEP,
                              "traffic_per_launch": measured_traffic(PER_LAYER_KERNEL, FIT_SOURCES,
                                                                     "fit_source_hash"),
                              "steps_per_launch": n_steps / 10.0},
            "per_layer_fp32_ms": out["per_layer_fp32"],
            "per_layer_fp32_steps_per_s": n_steps / (out["per_layer_fp32"] * 1e-3),
            "per_layer_fp32_hbm": {"bound": "hbm", "achieved": gbs32, "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": gbs32 / HBM_PEAK_GBS,
                                   "bytes_per_step": FIT_BYTES_PER_STEP}}


FIELD_Z0, FIELD_STEP = 300.0, 2.0


def tile_fit_set(ev, n_total, ms=10):
    """Step-major fit arrays of an event's tracks replicated at distinct
    addresses up to n_total (step k of track i is hit k*ld+i)."""
    ld = (n_total + 63) // 64 * 64
    m = ev.n_tracks
    bx = np.zeros((ms, m), np.float32)
    by, bz_ = np.zeros_like(bx), np.zeros_like(bx)
    bsu, bsv = np.full_like(bx, 0.01), np.full_like(bx, 0.05)
    bl = np.zeros((ms, m), np.int32)
    blseq = np.full((ms, m), -1, np.int32)
    for s in range(ms):
        hi = ev.seq_hit[:, s]
        msk = hi >= 0
        src = hi[msk]
        bx[s, msk], by[s, msk], bz_[s, msk] = ev.x[src], ev.y[src], ev.z[src]
        bsu[s, msk], bsv[s, msk], bl[s, msk] = ev.su[src], ev.sv[src], ev.layer[src]
        blseq[s, msk] = ev.seq_layer[msk, s]
    reps = (n_total + m - 1) // m

    def tile(a, fill):
        out = np.full((ms, ld), fill, a.dtype)
        out[:, :n_total] = np.tile(a, (1, reps))[:, :n_total]
        return out
    lseq = tile(blseq, -1)
    hits = dict(x=tile(bx, 0).reshape(-1), y=tile(by, 0).reshape(-1), z=tile(bz_, 0).reshape(-1),
                su=tile(bsu, 0.01).reshape(-1), sv=tile(bsv, 0.05).reshape(-1),
                layer=tile(bl, 0).reshape(-1))
    hidx = np.where(lseq >= 0, (np.arange(ms)[:, None] * ld + np.arange(ld)[None, :]), -1)
    return ld, hits, lseq, hidx.astype(np.int32)


def time_fused_fit(K, torch, ctx, ld, hits_np, lseq_np, hidx_np, n, flags=0, reps=5):
    """Mean kernel ms of kf_fit over n tracks (HIP events), seeding untimed."""
    hits = K.Hits(hits_np["x"], hits_np["y"], hits_np["z"], hits_np["su"], hits_np["sv"],
                  hits_np["layer"])
    lseq = torch.as_tensor(lseq_np, device="cuda")
    hidx = torch.as_tensor(hidx_np, device="cuda")
    seed_hits = hidx[:3].contiguous()
    t = K.Tracks(n, ld, flags & 3)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for r in range(-1, reps):
        ctx.seed(hits, seed_hits, t, flags & 3)
        if r >= 0:
            ev[r][0].record(stream)
        ctx.fit(t, hits, lseq, hidx, 10, flags=flags)
        if r >= 0:
            ev[r][1].record(stream)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in ev]))


def run_material(K, torch, steps, warmup, width, largest_first, n_fit):
    """The r-z material map with energy loss against constant per-layer
    material: the batched finding pass on a 64-event batch simulated with the
    map (scattering and energy loss), and the fused fit of n_fit tracks."""
    import eventgen as E
    import eventgen.material as EM
    from paper_1906_02253_amd import pipeline
    geom, mat, evs = EM.eloss_batch(seed=2)
    inp = E.find_inputs(evs)
    n_seeds = int(inp["seed_hits"].shape[0])
    out = {"workload": "64-event batch (seed 2) simulated with scattering and energy loss from an "
                       "r-z map (250 x 250 cells, ~0.02 X0 per surface); finding pass with the map "
                       "vs constant 0.02 X0 per layer without energy loss; fused fit of "
                       f"{n_fit} tracks (pT 0.5-1 GeV, ~0.05 X0) likewise",
           "n_seeds": n_seeds}
    for name, g, m in (("layer_x0", [dict(L, x0=0.02) for L in geom], None), ("map", geom, mat)):
        ctx = K.Context(g)
        ctx.set_find_config(width, largest_first)
        if m is not None:
            ctx.set_material(m)
        fp = pipeline.FindProblem(ctx, inp)
        ms, ph, cnt = timed_pass(torch, ctx, fp, 0, steps, warmup)
        kf = 3 * n_seeds + float(cnt[0])
        out["find_" + name] = {"ms_per_pass": ms, "steps_per_s": kf / (ms * 1e-3),
                               "find_kernel_ms": ph[3], "kf_steps_per_pass": kf}
    fgeom, fmat, fev = EM.eloss_sample(n_tracks=100_000, seed=24)
    ld, hits, lseq, hidx = tile_fit_set(fev, n_fit)
    n_steps = int((lseq[:, :n_fit] >= 0).sum())
    for name, g, m in (("layer_x0", [dict(L, x0=0.05) for L in fgeom], None), ("map", fgeom, fmat)):
        ctx = K.Context(g)
        if m is not None:
            ctx.set_material(m)
        ms = time_fused_fit(K, torch, ctx, ld, hits, lseq, hidx, n_fit)
        out["fit_" + name] = {"kernel_ms": ms, "steps_per_s": n_steps / (ms * 1e-3),
                              "kf_steps": n_steps}
    return out


def build_field_fit_set(n_total, n_unique=100_000, seed=7):
    """Fit sample in the parametrised field Bz = 3.8 T / (1 + (z/300 cm)^2)
    (pT U(0.5, 10) GeV, |eta| < 1, ten barrel layers, no material), traced
    with 0.5 cm Runge-Kutta steps: n_unique tracks replicated at distinct
    addresses up to n_total, hits step-major.  Also returns the unique
    tracks' layer-to-layer propagations (state at the crossing of layer k,
    layer k+1) for the evaluation counts."""
    import eventgen.field as EF
    geom, ev = EF.field_sample(n_tracks=n_unique, seed=seed, step=0.5)
    ld = (n_total + 63) // 64 * 64
    ms = 10
    m = n_unique
    bx = np.zeros((ms, m), np.float32)
    by, bz_ = np.zeros_like(bx), np.zeros_like(bx)
    bsu, bsv = np.full_like(bx, 0.01), np.full_like(bx, 0.05)
    bl = np.zeros((ms, m), np.int32)
    blseq = np.full((ms, m), -1, np.int32)
    for s in range(ms):
        hi = ev.seq_hit[:, s]
        msk = hi >= 0
        src = hi[msk]
        bx[s, msk], by[s, msk], bz_[s, msk] = ev.x[src], ev.y[src], ev.z[src]
        bsu[s, msk], bsv[s, msk], bl[s, msk] = ev.su[src], ev.sv[src], ev.layer[src]
        blseq[s, msk] = ev.seq_layer[msk, s]
    reps = (n_total + m - 1) // m

    def tile(a, fill):
        out = np.full((ms, ld), fill, a.dtype)
        out[:, :n_total] = np.tile(a, (1, reps))[:, :n_total]
        return out
    lseq = tile(blseq, -1)
    hits = dict(x=tile(bx, 0).reshape(-1), y=tile(by, 0).reshape(-1), z=tile(bz_, 0).reshape(-1),
                su=tile(bsu, 0.01).reshape(-1), sv=tile(bsv, 0.05).reshape(-1),
                layer=tile(bl, 0).reshape(-1))
    hidx = np.where(lseq >= 0, (np.arange(ms)[:, None] * ld + np.arange(ld)[None, :]), -1)
    nh = ev.n_track_hits()
    st, tg = [], []
    for k in range(ms - 1):
        msk = nh > k + 1
        st.append(ev.truth_at[msk, k])
        tg.append(np.full(int(msk.sum()), k + 1, np.int32))
    return geom, ld, hits, lseq, hidx.astype(np.int32), np.concatenate(st), np.concatenate(tg)


def field_flops_per_step(oc, evals, lengths):
    """Operations of one field propagation and update: the solve's set-up,
    each evaluation (its Runge-Kutta transport over the path taken as the
    converged one), the converged solve's polish step and state, the field
    transport of the covariance and the update; special-function calls
    counted as one.  evals and lengths are per-propagation arrays (3D path,
    cm)."""
    f = lambda k: oc[k]["ops"] + oc[k]["sfu"]
    n = np.ceil(np.abs(lengths) / FIELD_STEP)
    per = (f("field_setup") + f("field_at") + evals * (f("field_eval") + f("rk_fixed") + n * f("rk_step"))
           + f("field_final") + f("field_transport") + f("update"))
    return float(per.mean())


def run_field_fit(K, torch, n, oc, reps=5):
    """Fused fit of n tracks in the parametrised field, plain and learned
    start (network trained on the device on the field workload's
    propagations): kernel ms (HIP events), rates, Runge-Kutta evaluations per
    propagation, and the arithmetic roofline estimate."""
    import eventgen as E
    import eventgen.field as EF
    from paper_1906_02253_amd import learned
    geom, ld, hits_np, lseq_np, hidx_np, pst, ptg = build_field_fit_set(n)
    ctx = K.Context(geom, field_z0=FIELD_Z0, field_step=FIELD_STEP)
    g2, states, tl = EF.field_pairs(n_tracks=20_000, seed=6)
    ps = learned.PairSet(ctx, states, tl)
    tr, va, _ = learned.split_rows(ps.ok_rows, seed=6)
    learned.train(ctx, ps, tr, E.mlp_init(6), epochs=20, batch=4096, lr=1e-3, seed=6)
    val = learned.eval_loss(ctx, ps, va)
    hits = K.Hits(hits_np["x"], hits_np["y"], hits_np["z"], hits_np["su"], hits_np["sv"],
                  hits_np["layer"])
    lseq = torch.as_tensor(lseq_np, device="cuda")
    hidx = torch.as_tensor(hidx_np, device="cuda")
    seed_hits = hidx[:3].contiguous()
    t = K.Tracks(n, ld)
    n_steps = int((lseq_np[:, :n] >= 0).sum())
    stream = torch.cuda.current_stream()
    out = {}
    for name, flags in (("plain", 0), ("learned", K.INIT_MLP)):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for r in range(-1, reps):
            ctx.seed(hits, seed_hits, t)
            if r >= 0:
                ev[r][0].record(stream)
            ctx.fit(t, hits, lseq, hidx, 10, flags=flags)
            if r >= 0:
                ev[r][1].record(stream)
        torch.cuda.synchronize()
        out[name] = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    cs = learned.compare_starts(ctx, pst, ptg)
    ok = cs["plain"]["status"] == 0
    l3 = cs["plain"]["path"][ok] / np.sin(pst[ok, 5])
    rep = {"workload": f"fit of {n} tracks in the field Bz = 3.8 T / (1 + (z/300 cm)^2), "
                       f"pT U(0.5,10) GeV, |eta|<1, 10 barrel layers, RK4 step <= 2 cm, mixed "
                       f"precision",
           "kf_steps": n_steps, "network_validation_loss": val}
    for name in ("plain", "learned"):
        it = cs[name]["iters"][ok].astype(np.float64)
        fl = field_flops_per_step(oc, it, l3) * n_steps
        tf = fl / (out[name] * 1e-3) / 1e12
        rep[name] = {"kernel_ms": out[name], "steps_per_s": n_steps / (out[name] * 1e-3),
                     "rk_evals_per_propagation": float(it.mean()),
                     "roofline_estimate": {"bound": "alu", "achieved": tf,
                                           "peak": VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                                           "frac": tf / VECTOR_PEAK_TFLOPS,
                                           "flops_per_launch": fl}}
    return rep


def run_field_find(K, torch, steps, warmup, width, largest_first):
    """The batched finding pass on field-traced events (16 events, N ~
    Poisson(U(200, 4000)) tracks, 60 noise hits per track, ten barrels) in the
    parametrised field, next surface by the Runge-Kutta radius solve; beside
    it the same events found with the uniform central field (the closed-form
    helix): ms per pass, KF steps/s, the finding kernel, solve evaluations per
    propagation and the hits found."""
    import eventgen as E
    import eventgen.field as EF
    from paper_1906_02253_amd import pipeline
    geom, evs = EF.field_find_batch()
    inp = E.find_inputs(evs)
    n_seeds = int(inp["seed_hits"].shape[0])
    out = {"workload": "16 events traced in Bz = 3.8 T / (1 + (z/300 cm)^2) (0.5 cm RK4 steps), "
                       "N ~ Poisson(U(200,4000)), pT U(0.5,10) GeV, |eta|<1, 60 noise hits/track, "
                       "10 barrel layers, no material; RK4 step <= 2 cm in the finder",
           "n_seeds": n_seeds, "n_hits": int(inp["x"].shape[0]), "width": width}
    for name, kw in (("field", dict(field_z0=FIELD_Z0, field_step=FIELD_STEP)), ("uniform", {})):
        ctx = K.Context(geom, **kw)
        ctx.set_find_config(width, largest_first)
        fp = pipeline.FindProblem(ctx, inp)
        ms, ph, cnt = timed_pass(torch, ctx, fp, 0, steps, warmup)
        h = fp.out_hits[:n_seeds].cpu().numpy()
        out[name] = {"ms_per_pass": ms, "steps_per_s": (3 * n_seeds + cnt[0]) / (ms * 1e-3),
                     "find_kernel_ms": ph[3], "kf_steps_per_pass": 3 * n_seeds + float(cnt[0]),
                     "solve_evals_per_propagation": float(cnt[3] / max(cnt[0], 1.0)),
                     "hits_found": int((h >= 0).sum())}
        del fp, ctx
    return out


LARGE_COPIES = 8


def run_large_find(K, torch, oc, geom, evs, steps, warmup, width, largest_first):
    """The batched finding pass over the batch replicated LARGE_COPIES times
    at distinct addresses (512 events, a working set of several GB, far above
    the 256 MB Infinity Cache): ms per pass, KF steps/s, the phases and the
    finding kernel's HBM roofline."""
    import eventgen as E
    from paper_1906_02253_amd import pipeline
    big = list(evs) * LARGE_COPIES
    inp = E.find_inputs(big)
    n_seeds = int(inp["seed_hits"].shape[0])
    n_hits = int(inp["x"].shape[0])
    ctx = K.Context(geom)
    ctx.set_find_config(width, largest_first)
    fp = pipeline.FindProblem(ctx, inp)
    ms, ph, cnt = timed_pass(torch, ctx, fp, 0, steps, warmup)
    kf = 3 * n_seeds + float(cnt[0])
    out = {"workload": f"batched finding over {len(big)} events: the 64-event batch replicated "
                       f"{LARGE_COPIES} times at distinct addresses",
           "n_events": len(big), "n_seeds": n_seeds, "n_hits": n_hits,
           "hit_input_bytes": n_hits * 24, "binned_hit_bytes": n_hits * 32, "width": width,
           "ms_per_pass": ms, "steps_per_s": kf / (ms * 1e-3), "kf_steps_per_pass": kf,
           "phases_ms": {"seed_and_seed_fit": ph[0], "binning": ph[1], "seed_order": ph[2],
                         "find_kernel": ph[3]},
           "roofline": find_roofline(cnt, ph[3], oc, None, FIND_KERNEL)}
    del fp, ctx
    return out


def run_clean_pass(K, torch, steps, warmup, width, largest_first):
    """The batched pass on the 64-event batch with module-overlap duplicate
    seeds (overlap hits at 10% per barrel and 30% per disk crossing on each
    track's first three layers, one seed per hit combination), without and
    with seed cleaning and duplicate removal of the found tracks (its time is
    inside the finding phase): ms per pass, the phases, seeds searched and
    tracks kept."""
    import eventgen.overlap as EO
    from paper_1906_02253_amd import pipeline
    geom, evs, ovls = EO.overlap_batch(seed=9)
    inp = EO.overlap_inputs(evs, ovls)
    n_seeds = int(inp["seed_hits"].shape[0])
    n_particles = int(np.unique(inp["seed_event"].astype(np.int64) * 1_000_000
                                + inp["seed_track"]).size)
    ctx = K.Context(geom)
    ctx.set_find_config(width, largest_first)
    fp = pipeline.FindProblem(ctx, inp)
    out = {"workload": "64-event batch (seed 9) with module-overlap duplicate seeds: overlap hits "
                       "at 10% per barrel and 30% per disk crossing on the first three layers, one "
                       "seed per combination of those hits",
           "n_seeds": n_seeds, "n_particles_seeded": n_particles, "width": width}
    for name, flags in (("no_cleaning", 0), ("cleaning", K.CLEAN_SEEDS),
                        ("duplicate_removal", K.REMOVE_DUPLICATES),
                        ("cleaning_and_duplicate_removal", K.CLEAN_SEEDS | K.REMOVE_DUPLICATES)):
        ms, (ms_seed, ms_bin, ms_order, ms_kernel), cnt = timed_pass(torch, ctx, fp, flags, steps,
                                                                     warmup)
        st = fp.out.status[:n_seeds].cpu().numpy()
        out[name] = {"ms_per_pass": ms, "seeds_per_s": n_seeds / (ms * 1e-3),
                     "phases_ms": {"seed_and_seed_fit": ms_seed, "binning": ms_bin,
                                   "seed_order_and_cleaning": ms_order,
                                   "find_kernel": ms_kernel},
                     "seeds_searched": int(((st & K.ST_DUPLICATE) == 0).sum()),
                     "tracks_kept": int(((st & (K.ST_DUPLICATE | K.ST_DUPTRACK)) == 0).sum()),
                     "kf_steps_per_pass": 3 * n_seeds + float(cnt[0])}
    out["cleaning_ms"] = (out["cleaning"]["phases_ms"]["seed_order_and_cleaning"]
                          - out["no_cleaning"]["phases_ms"]["seed_order_and_cleaning"])
    out["speedup"] = out["no_cleaning"]["ms_per_pass"] / out["cleaning"]["ms_per_pass"]
    out["duplicate_removal_ms"] = (out["duplicate_removal"]["phases_ms"]["find_kernel"]
                                   - out["no_cleaning"]["phases_ms"]["find_kernel"])
    return out


def copy_probe(torch, mib=1024, reps=5):
    """A plain streaming kernel of known size (read mib MiB, write mib MiB):
    its bandwidth, and the reference the HBM byte counters are scaled by."""
    x = torch.ones(mib * 2 ** 18, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.mul(x, 2.0, out=y)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        torch.mul(x, 2.0, out=y)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    return {"bytes": 2 * mib * 2 ** 20, "ms": ms, "gbs": 2 * mib * 2 ** 20 / (ms * 1e-3) / 1e9}


def timed_pass(torch, ctx, fp, flags, steps, warmup):
    """Warm-up, then `steps` replays of the captured finding pass; returns
    (wall ms per pass, mean phase ms (seed fit, binning, seed order, finding
    kernel) from the HIP events inside the graph, counters per pass)."""
    for _ in range(warmup):
        fp.run_batched(flags)
    torch.cuda.synchronize()
    c0 = fp.counters.clone()
    ctx.set_timing(steps)
    torch.cuda.synchronize()
    start = time.perf_counter()
    for _ in range(steps):
        fp.run_batched(flags)
    torch.cuda.synchronize()
    wall = time.perf_counter() - start
    phases, _ = ctx.timings()
    ctx.set_timing(0)
    cnt = ((fp.counters - c0).double() / steps).cpu().numpy()
    return wall * 1e3 / steps, phases, cnt


def train_guess(K, torch, E, workload):
    """Trains the learned start on the device: 1e6 pairs from the plain
    propagator at the distribution it will serve ("batch": the finding batch's
    states at every surface paired with the next barrel outward, drawn from
    64 events of their own; "precision": the fit throughput set's barrel
    hops), 20 epochs of batch 4096, Adam 1e-3.  Returns (weights, report)."""
    from paper_1906_02253_amd import learned
    t0 = time.time()
    if workload == "batch":
        geom, states, tl = E.batch_propagation_pairs(n_pairs=1_000_000, seed=5)
    else:
        geom, states, tl = E.propagation_pairs(n_pairs=1_000_000, seed=4)
    ctx = K.Context(geom)
    ps = learned.PairSet(ctx, states, tl)
    tr, va, te = learned.split_rows(ps.ok_rows, seed=4)
    torch.cuda.synchronize()
    t_data = time.time() - t0
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    losses = learned.train(ctx, ps, tr, E.mlp_init(4), epochs=20, batch=4096, lr=1e-3, seed=4)
    b.record()
    torch.cuda.synchronize()
    train_ms = a.elapsed_time(b)
    val = learned.eval_loss(ctx, ps, va)
    r = learned.compare_starts(ctx, states[te], tl[te])
    ok = r["plain"]["status"] == 0
    it_p, it_l = r["plain"]["iters"][ok], r["learned"]["iters"][ok]
    n_steps = losses.shape[0]
    rep = {"workload": workload, "pairs": int(ps.n), "train_rows": int(tr.size), "epochs": 20, "batch": 4096,
           "adam_steps": int(n_steps), "train_ms": train_ms,
           "train_rows_per_s": n_steps * 4096 / (train_ms * 1e-3),
           "train_tflops": n_steps * 4096 * 3 * 2 * 4672 / (train_ms * 1e-3) / 1e12,
           "final_train_loss": float(losses[-50:].mean()), "validation_loss": val,
           "held_out_propagations": int(ok.sum()),
           "r_evals_plain_mean": float(it_p.mean()), "r_evals_plain_p99": float(np.percentile(it_p, 99)),
           "r_evals_learned_mean": float(it_l.mean()),
           "r_evals_learned_p99": float(np.percentile(it_l, 99)),
           "data_prep_s": t_data}
    return ctx.mlp_get(), rep


def oracle_find_all(oracle, geom, evs, inp, threads):
    """The FP64 oracle's seed fit + finding over every event; returns its
    propagation count."""
    cfg = oracle.Config(geom)
    n_prop = 0
    for e, ev in enumerate(evs):
        m = np.nonzero(inp["seed_event"] == e)[0]
        if m.size:
            n_prop += oracle.find(cfg, ev, inp["seed_hits_local"][m], n_threads=threads)["n_prop"]
    return n_prop


def cpu_model():
    """The host CPU's model name (lscpu), or '' where it cannot be read."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return ""
    for line in out.splitlines():
        if line.startswith("Model name:"):
            return line.split(":", 1)[1].strip()
    return ""


def cpu_baseline(geom, evs, inp, single_events=64):
    """The FP64 oracle's seed fit and finding timed on the host: over the
    whole batch on all host threads (capped at 16, the host share one GPU
    gets), and over its first `single_events` events on one thread."""
    import oracle
    threads = min(os.cpu_count() or 1, 16)
    n_seeds = int(inp["seed_hits"].shape[0])
    c0 = time.perf_counter()
    n_prop = oracle_find_all(oracle, geom, evs, inp, threads)
    cdt = time.perf_counter() - c0
    csteps = 3 * n_seeds + n_prop
    sub = evs[:single_events]
    n_sub = int((inp["seed_event"] < single_events).sum())
    c1 = time.perf_counter()
    n_prop1 = oracle_find_all(oracle, geom, sub, inp, 1)
    c1dt = time.perf_counter() - c1
    s1 = 3 * n_sub + n_prop1
    return {"value": csteps / cdt, "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle seed fit + finding over the same 64-event batch on {threads} "
                      f"threads: {csteps} KF steps in {cdt:.2f} s",
            "single_thread": {"value": s1 / c1dt, "unit": "steps/s", "cores": 1,
                              "sample": f"the batch's first {single_events} events on one "
                                        f"thread: {s1} KF steps in {c1dt:.2f} s"},
            "host_threads": os.cpu_count(), "cpu_model": cpu_model()}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: events are independent, the path shards by event "
              "with no exchange, and the library drives one GPU per process; use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import eventgen as E
    import paper_1906_02253_amd as K
    from paper_1906_02253_amd import pipeline
    from paper_1906_02253_amd.build import OPCOUNT_JSON

    with open(OPCOUNT_JSON) as f:
        oc = json.load(f)
    torch.cuda.set_device(0)
    t0 = time.time()
    geom, evs = E.batch_events()
    inp = E.find_inputs(evs)
    n_seeds = int(inp["seed_hits"].shape[0])
    print(f"# batch: {len(evs)} events, {n_seeds} seeds, {inp['x'].shape[0]} hits "
          f"({time.time() - t0:.1f} s)", file=sys.stderr, flush=True)

    probe = copy_probe(torch)
    ctx = K.Context(geom)
    fp = pipeline.FindProblem(ctx, inp)
    fp.run()
    tune = None
    if args.width:
        ctx.set_find_config(args.width, args.largest_first)
    else:
        tune = fp.autotune(reps=3)
        print("# autotune (width, largest_first) -> ms: " +
              ", ".join(f"{w}/{int(lf)}: {ms:.3f}" for (w, lf), ms in sorted(tune.items())),
              file=sys.stderr, flush=True)
    width, largest_first = ctx.find_config()
    # the timed pass: seeding, seed fit, binning, seed order and the finding
    # kernel replayed as one captured graph
    ms_per_step, (ms_seed, ms_bin, ms_sort, ms_kernel), cnt = timed_pass(
        torch, ctx, fp, 0, args.steps, args.warmup)
    kf_steps = 3 * n_seeds + cnt[0]
    value = kf_steps / (ms_per_step * 1e-3)
    roof = find_roofline(cnt, ms_kernel, oc, measured_traffic(FIND_KERNEL), FIND_KERNEL)
    print(f"# {ms_per_step:.3f} ms/step, find kernel {ms_kernel:.3f} ms, seed+fit {ms_seed:.3f} ms, "
          f"binning {ms_bin:.3f} ms, seed order {ms_sort:.3f} ms, {kf_steps:.0f} KF steps/pass",
          file=sys.stderr, flush=True)

    result = {
        "metric": "KF prop+update steps/s",
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 storage, f32+f64 arithmetic",
        "data": "synthetic",
        "config": {"workload": "batched finding: 64 events, N ~ Poisson(U(200,4000)), 60 noise "
                               "hits/track, 10 barrel layers + 2x7 disks, |eta|<2.5, 0.02 X0, "
                               "chi2<30, <=6 candidates/seed; seed + seed fit + kf_find",
                   "n_events": len(evs), "n_seeds": n_seeds, "n_hits": int(inp["x"].shape[0]),
                   "kf_steps_per_pass": kf_steps, "width": width,
                   "tile_order": "largest events first" if largest_first else "event, eta, phi",
                   "autotune_ms": {f"{w}/{int(lf)}": ms for (w, lf), ms in sorted(tune.items())}
                   if tune else None,
                   "launch": "hipGraph replay (kf_find_batched)",
                   "precision": "mixed (FP32 storage, FP64 covariance arithmetic and update)",
                   "init": "plain"},
        "roofline": roof,
        "phases_ms": {"seed_and_seed_fit": ms_seed, "binning": ms_bin, "seed_order": ms_sort,
                      "find_kernel": ms_kernel},
        "copy_probe": probe,
    }

    if not args.no_large:
        result["find_large"] = run_large_find(K, torch, oc, geom, evs, args.steps, args.warmup,
                                              width, largest_first)
        fl = result["find_large"]
        print(f"# {fl['n_events']} events: {fl['ms_per_pass']:.3f} ms/pass "
              f"({fl['steps_per_s']:.3e} steps/s), find kernel {fl['phases_ms']['find_kernel']:.3f} "
              f"ms, {fl['roofline']['achieved']:.0f} GB/s by the model", file=sys.stderr, flush=True)

    # learned start: train on the device, then the same timed pass
    w, rep = train_guess(K, torch, E, "batch")
    ctx.mlp_load(w)
    if width < 64:
        ctx.set_find_config(64, largest_first)
    ms_l, ph_l, cnt_l = timed_pass(torch, ctx, fp, K.INIT_MLP, args.steps, args.warmup)
    steps_l = 3 * n_seeds + cnt_l[0]
    rep.update({"steps_per_s": steps_l / (ms_l * 1e-3), "ms_per_step": ms_l,
                "find_kernel_ms": ph_l[3], "kf_steps_per_pass": steps_l,
                "r_evals_per_propagation_plain": cnt[3] / cnt[0],
                "r_evals_per_propagation_learned": cnt_l[3] / cnt_l[0],
                "guesses_per_pass": cnt_l[5], "fallbacks_per_pass": cnt_l[6],
                "fallback_rate": cnt_l[6] / max(cnt_l[5], 1.0),
                "mlp_tflops_in_find": cnt_l[5] * 2 * 4672 / (ph_l[3] * 1e-3) / 1e12})
    result["learned_init"] = rep
    print(f"# learned start: {ms_l:.3f} ms/step ({rep['steps_per_s']:.3e} steps/s), find kernel "
          f"{ph_l[3]:.3f} ms; r(s) evaluations per propagation {cnt[3] / cnt[0]:.3f} plain, "
          f"{cnt_l[3] / cnt_l[0]:.3f} learned; training {rep['train_ms']:.1f} ms",
          file=sys.stderr, flush=True)

    # steering: the same batch and pass following the five-region layer plans
    sctx = K.Context(geom)
    sctx.set_find_config(width, largest_first)
    sctx.set_steering(E.geometry.steering_plans(geom))
    sfp = pipeline.FindProblem(sctx, inp)
    ms_s, ph_s, cnt_s = timed_pass(torch, sctx, sfp, 0, args.steps, args.warmup)
    fp.run_batched(0)                   # the dynamic navigation's hit lists, plain start
    torch.cuda.synchronize()
    fp_hits = fp.out_hits[:n_seeds].cpu().numpy()
    s_hits = sfp.out_hits[:n_seeds].cpu().numpy()
    result["steering"] = {
        "plans": "five eta regions (|eta| < 0.8, 0.8-1.6, 1.6-2.5, both signs), each the layers a "
                 "straight line from the origin crosses, ordered by path length",
        "ms_per_step": ms_s, "steps_per_s": (3 * n_seeds + cnt_s[0]) / (ms_s * 1e-3),
        "find_kernel_ms": ph_s[3], "kf_steps_per_pass": 3 * n_seeds + float(cnt_s[0]),
        "hits_found": int((s_hits >= 0).sum()), "hits_found_dynamic": int((fp_hits >= 0).sum()),
        "identical_hit_lists": float((s_hits == fp_hits).all(axis=1).mean())}
    print(f"# steering: {ms_s:.3f} ms/step, find kernel {ph_s[3]:.3f} ms; hits found "
          f"{result['steering']['hits_found']} vs {result['steering']['hits_found_dynamic']} dynamic",
          file=sys.stderr, flush=True)
    del sfp, sctx

    if not args.no_fit:
        w_fit, rep_fit = train_guess(K, torch, E, "precision")
        result["fit"] = run_fit(K, torch, args.fit_tracks, w_fit)
        result["fit"]["learned_training"] = rep_fit
        print(f"# fit: {result['fit']['fused_steps_per_s']:.3e} steps/s fused", file=sys.stderr,
              flush=True)

    if not args.no_fit:
        result["field_fit"] = run_field_fit(K, torch, args.field_tracks, oc)
        ff = result["field_fit"]
        print(f"# field fit: {ff['plain']['steps_per_s']:.3e} steps/s plain, "
              f"{ff['learned']['steps_per_s']:.3e} learned; RK evaluations per propagation "
              f"{ff['plain']['rk_evals_per_propagation']:.3f} / "
              f"{ff['learned']['rk_evals_per_propagation']:.3f}", file=sys.stderr, flush=True)

    if not args.no_field_find:
        result["field_find"] = run_field_find(K, torch, args.steps, args.warmup, width,
                                              largest_first)
        ff = result["field_find"]
        print(f"# field find: {ff['field']['ms_per_pass']:.3f} ms/pass "
              f"({ff['field']['steps_per_s']:.3e} steps/s), uniform field "
              f"{ff['uniform']['ms_per_pass']:.3f} ms; hits found {ff['field']['hits_found']} vs "
              f"{ff['uniform']['hits_found']}", file=sys.stderr, flush=True)

    if not args.no_clean:
        result["seed_cleaning"] = run_clean_pass(K, torch, args.steps, args.warmup, width,
                                                 largest_first)
        sc = result["seed_cleaning"]
        print(f"# seed cleaning: {sc['n_seeds']} seeds -> {sc['cleaning']['seeds_searched']} "
              f"searched; pass {sc['no_cleaning']['ms_per_pass']:.3f} -> "
              f"{sc['cleaning']['ms_per_pass']:.3f} ms (cleaning {sc['cleaning_ms']:.3f} ms)",
              file=sys.stderr, flush=True)

    if not args.no_material:
        result["material_map"] = run_material(K, torch, args.steps, args.warmup, width,
                                              largest_first, 1_000_000)
        mm = result["material_map"]
        print(f"# material map: find pass {mm['find_layer_x0']['ms_per_pass']:.3f} -> "
              f"{mm['find_map']['ms_per_pass']:.3f} ms; fit {mm['fit_layer_x0']['steps_per_s']:.3e} "
              f"-> {mm['fit_map']['steps_per_s']:.3e} steps/s", file=sys.stderr, flush=True)

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(geom, evs, inp)
        cb = result["cpu_baseline"]
        print(f"# cpu oracle: {cb['value']:.3e} steps/s on {cb['cores']} threads, "
              f"{cb['single_thread']['value']:.3e} on one ({cb['cpu_model']})", file=sys.stderr,
              flush=True)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
