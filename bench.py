"""Benchmark: MPPI control steps per second on one MI355X.

One benchmark step = one MPPI control step of Algorithm 1 on the device: one
iteration (noise, rollouts with the likelihood-ratio cost, min-shifted weights, FP64
normaliser and weighted update), emission of u0, the warm shift, and the harness
plant step, with the state and the emitted control resident in HBM.  The timed
region runs these steps back to back as a closed loop on the device, ten steps per
launch sequence (one captured graph; --steps-per-launch), which removes the gap the
runtime leaves between consecutive graph launches; `value` is rollout-steps per second
(K * T * iterations / wall time).  The rate with one launch per control step (what a
loop that waits for each external state measurement sees) is reported beside it.

Default workload: the kinematic bicycle on a 256 x 256 cost map, K = 4096, T = 100,
nu = 2.  Other single-GPU workloads can be chosen with --workload.

The JSON line also carries the dominant kernel's roofline (its mean duration from
HIP events recorded on the library's own stream during a profiled pass of the same
length), the serving legs (a Poisson trace at 50 Hz per controller and a saturated
burst, batched against one controller at a time) and the CPU leg: the oracle's
throughput on a bounded sample of the same workload, plus one control step of the
timed controller checked against the oracle.  Only the CPU leg touches the oracle.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rollout-steps/sec (K*T) and MPPI iters/sec; p50/p99 step latency batched vs plain"

# Algorithmic operations per rollout-step of the rollout kernel (FMA = 2, every other
# FP32/FP64 arithmetic op, transcendental and Philox integer op = 1), counted per part:
# noise (a quarter of a Philox4x32-10 call with its uniforms and Box-Muller per control,
# about 130 ops per call), du = A L eps and v = u + du, the dynamics, the Euler update,
# the state cost and the likelihood-ratio control terms; for example the quadrotor:
# 130 + 24 + 80 + 24 + 428 (32 obstacles x 13 + goal) + 54 = 740.
ALG_OPS_PER_ROLLOUT_STEP = {"cartpole": 87, "bicycle": 164, "quadrotor": 740, "linear": 90,
                            "cartpole_swingup": 77, "quadrotor_crash": 1064,
                            "bicycle_ctg": 164}     # same arithmetic; the prefix costs are stores
# MLP [16 -> 128 -> 128 -> 12]: 2 (16*128 + 128*128 + 128*12) FLOP per rollout-step on BF16 MFMA.
MLP_FLOP_PER_ROLLOUT_STEP = 2 * (16 * 128 + 128 * 128 + 128 * 12)
BF16_MFMA_PEAK_TFLOPS = 2500.0

# VALU peak without packed FP32 (the build forbids v_pk_*_f32): 256 CUs x 4 SIMD x 16 lanes
# x 2 (FMA) x 2.4 GHz.
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PUBLISHED_FP32_TFLOPS = 157.3


TRAFFIC_FILES = {"bicycle": "traffic_rollout_bicycle_K4096_T100.md",
                 "quadrotor": "traffic_rollout_quadrotor_K16384_T150.md"}
ROLLOUT_SOURCES = ["mppi_device.h", "mppi_systems.h", "mppi_kernels.h"]


def measured_traffic(name):
    """HBM bytes per rollout launch from the committed rocprofv3 counter summary (FETCH_SIZE and
    WRITE_SIZE, each divided by its factor on a known-size copy), or None when there is none or
    the rollout kernel's sources have changed since the counters were taken."""
    import hashlib
    fn = TRAFFIC_FILES.get(name)
    path = os.path.join(ROOT, "profiles", fn) if fn else None
    if not path or not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", " ", "`")):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in ROLLOUT_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1509_01149_amd", "csrc", f), "rb").read())
    if rec.get("kernel_source_sha256") != h.hexdigest():
        return None
    return int(rec["traffic_bytes_per_launch"])


def make_workload(name):
    import workloads as W
    if name == "bicycle":
        return W.bicycle().replace(seed=0)
    if name == "cartpole":
        return W.cartpole(nu=2.0).replace(seed=0)
    if name == "quadrotor":
        return W.quadrotor(nu=2.0).replace(seed=0)
    if name == "quadrotor_crash":
        return W.quadrotor(nu=2.0, crash=True).replace(seed=0, name="quadrotor_crash")
    if name == "bicycle_ctg":               # the bicycle under cost-to-go weighting
        return W.bicycle().replace(seed=0, name="bicycle_ctg")
    if name == "swingup":
        return W.cartpole_swingup(nu=1000.0, K=4096).replace(seed=0)
    if name == "quadrotor_mlp":
        return W.quadrotor_mlp(trained_mlp(), nu=2.0, K=16384, T=100).replace(seed=0)
    raise SystemExit(f"unknown workload {name}")


def trained_mlp(n=1_000_000, epochs=20):
    """The learned-dynamics network, trained on the GPU on n analytic transitions."""
    import workloads as W
    import paper_1509_01149_amd as P
    wl = W.quadrotor()
    x, u = W.mlp_training_inputs(n)
    g = P.Mlp(W.mlp_init_weights())
    g.set_dataset(wl.params, wl.dt, x, u)
    t0 = time.perf_counter()
    for ep, order in enumerate(W.minibatch_order(n, epochs)):
        losses = g.train(order, 4096, 2e-3 * 0.5 ** (ep // 5))
    g.train_seconds = time.perf_counter() - t0
    g.final_loss = float(losses.mean())
    return g


def serving_mix_workloads(n_controllers):
    import workloads as W
    out = []
    for i, (sysid, K, T) in enumerate(W.serving_mix(n_controllers)):
        if sysid == 0:
            wl = W.cartpole(nu=2.0, K=K, T=T)
        elif sysid == 1:
            wl = W.bicycle(K=K, T=T)
        else:
            wl = W.quadrotor(nu=2.0, K=K, T=T)
        out.append(wl.replace(seed=1000 + i))
    return out


def serving_bench(seconds, plain_seconds, n_controllers=256, rate_hz=50.0, inflight=3, saturate_requests=8):
    """Replay the same Poisson trace (rate_hz per controller) through the batched server
    and through the plain one-controller-at-a-time policy; report latency percentiles and
    aggregate rollout-steps/s."""
    import workloads as W
    import paper_1509_01149_amd as P
    wls = serving_mix_workloads(n_controllers)
    trace = W.poisson_arrivals(n_controllers, rate_hz, max(seconds, plain_seconds))
    res = dict(controllers=n_controllers, rate_hz_per_controller=rate_hz,
               offered_requests_per_s=n_controllers * rate_hz,
               offered_rollout_steps_per_s=rate_hz * sum(w.K * w.T for w in wls))
    for mode, dur in (("batched", seconds), ("plain", plain_seconds)):
        if dur <= 0:
            continue
        ev = [(t, c) for t, c in trace if t < dur]
        t = np.array([a for a, _ in ev])
        ci = np.array([c for _, c in ev])
        kw = dict(max_slots=n_controllers, max_inflight=inflight, max_batch=n_controllers,
                  mode=P.SERVE_BATCHED if mode == "batched" else P.SERVE_PLAIN, hbm_budget_bytes=64 << 30)
        with P.Server(**kw) as srv:
            slots = np.array([srv.admit(**P.controller_args(wl)) for wl in wls])
            # warm up: one request per controller, not timed
            srv.replay(np.zeros(n_controllers), slots, [np.pad(w.x0, (0, 16 - w.n)) for w in wls])
            st0 = srv.stats()
            x0s = [np.pad(wls[c].x0, (0, 16 - wls[c].n)) for c in ci]
            td, u0, status = srv.replay(t, slots[ci], x0s)
            st1 = srv.stats()
        lat = (td - t) * 1e3
        span = float(td.max())
        steps = float(sum(wls[c].K * wls[c].T for c in ci))
        res[mode] = dict(trace_seconds=dur, requests=int(t.size), p50_ms=round(float(np.percentile(lat, 50)), 3),
                         p99_ms=round(float(np.percentile(lat, 99)), 3), max_ms=round(float(lat.max()), 3),
                         mean_ms=round(float(lat.mean()), 3), completion_span_s=round(span, 3),
                         rollout_steps_per_s=round(steps / span, 1), requests_per_s=round(t.size / span, 1),
                         mean_batch=round((st1["batches"] and (st1["requests_done"] - st0["requests_done"]) /
                                           max(1, st1["batches"] - st0["batches"])), 2),
                         numeric_failures=int(np.sum(status != 0)))
    if saturate_requests > 0:
        res["saturated"] = saturation_bench(wls, saturate_requests, inflight)
    return res


def saturation_bench(wls, per_controller, inflight):
    """Capacity: every controller's requests arrive at once (per_controller each, served in
    order, at most one in flight per controller), through both policies; the completion
    span gives the sustained rate when the queue never empties."""
    import paper_1509_01149_amd as P
    n = len(wls)
    ci = np.tile(np.arange(n), per_controller)
    t = np.zeros(ci.size)
    steps = float(sum(wls[c].K * wls[c].T for c in ci))
    ops = float(sum(ALG_OPS_PER_ROLLOUT_STEP[wls[c].name] * wls[c].K * wls[c].T for c in ci))
    out = dict(requests_per_controller=per_controller, requests=int(ci.size))
    for mode in ("batched", "plain"):
        kw = dict(max_slots=n, max_inflight=inflight, max_batch=n,
                  mode=P.SERVE_BATCHED if mode == "batched" else P.SERVE_PLAIN, hbm_budget_bytes=64 << 30)
        with P.Server(**kw) as srv:
            slots = np.array([srv.admit(**P.controller_args(wl)) for wl in wls])
            srv.replay(np.zeros(n), slots, [np.pad(w.x0, (0, 16 - w.n)) for w in wls])
            st0 = srv.stats()
            td, _, status = srv.replay(t, slots[ci], [np.pad(wls[c].x0, (0, 16 - wls[c].n)) for c in ci])
            st1 = srv.stats()
        span = float(td.max())
        out[mode] = dict(completion_span_s=round(span, 4), requests_per_s=round(ci.size / span, 1),
                         rollout_steps_per_s=round(steps / span, 1),
                         rollout_alg_tflops=round(ops / span / 1e12, 3),
                         frac_of_alu_peak=round(ops / span / 1e12 / ALU_PEAK_TFLOPS, 4),
                         mean_batch=round((st1["requests_done"] - st0["requests_done"]) /
                                          max(1, st1["batches"] - st0["batches"]), 2),
                         numeric_failures=int(np.sum(status != 0)))
    out["batched_over_plain"] = round(out["plain"]["completion_span_s"] / out["batched"]["completion_span_s"], 2)
    return out


def cpu_baseline(wl, seconds):
    """The FP64 oracle, as it stands, on a bounded closed-loop sample of the workload."""
    from oracle import mppi
    x = np.asarray(wl.x0, float).copy()
    U = mppi.initial_sequence(wl)
    it = 0
    t0 = time.perf_counter()
    while True:
        u0, U, it, _ = mppi.control_step(wl, x, U, it)
        x = mppi.plant_step(wl, x, u0)
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return dict(value=wl.K * wl.T * it / el, unit="rollout-steps/s", cores=1, kind="oracle",
                sample=f"{it} closed-loop control steps of the same workload (K={wl.K}, T={wl.T}), "
                       f"{el:.1f} s, NumPy FP64 on one host thread")


def parity_spot_check(wl, ctrl, x):
    """One control step of the timed controller against the oracle's, from the same state,
    nominal sequence and iteration (part of the CPU leg)."""
    from oracle import mppi
    U = ctrl.get_controls()
    it = ctrl.iteration()
    u0 = ctrl.step(x)
    U_gpu = ctrl.get_controls()
    u0_r, U_r, _, _ = mppi.control_step(wl, x, U, it)
    scale = max(1.0, float(np.max(np.abs(U_r))))
    return dict(U_rel_err=float(max(np.max(np.abs(U_gpu - U_r)), np.max(np.abs(u0 - u0_r))) / scale),
                tolerance=1e-4, at_iteration=it)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--steps-per-launch", type=int, default=10,
                    help="closed-loop steps per launch sequence (captured graph); 1 = one launch per step")
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--workload", default="bicycle")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--serving-seconds", type=float, default=2.0,
                    help="length of the batched serving trace (0 disables the serving leg)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="first run one plain device copy of this many bytes (a known-size kernel for "
                         "calibrating HBM byte counters in a profiler pass)")
    ap.add_argument("--plain-seconds", type=float, default=1.0,
                    help="length of the same trace replayed one controller at a time")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the MPPI path shards over samples with one small "
              f"exchange per iteration, which is designed but not built; --gpus {args.gpus} is not supported.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1509_01149_amd as P
    P.load()
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible: bench.py runs the HIP path only")
    dev = torch.device("cuda:0")
    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    wl = make_workload(args.workload)
    stream = torch.cuda.current_stream(dev)
    ctg = wl.name.endswith("_ctg")
    ctrl = P.controller_for(wl, device=0, torch_stream=stream, torch_workspace=True,
                            **(dict(weighting=P.WEIGHT_COST_TO_GO) if ctg else {}))
    x_dev = torch.tensor(np.asarray(wl.x0, float), dtype=torch.float64, device=dev)
    spl = max(1, args.steps_per_launch)
    u_log = torch.zeros((spl, wl.m), dtype=torch.float64, device=dev)
    xp, up = x_dev.data_ptr(), u_log.data_ptr()

    def run(n, per_launch=spl):
        """n closed-loop control steps on the device, per_launch steps per launch sequence
        (one captured graph each); every step is the whole path: rollout, update, finalize
        with emit, shift and the plant step."""
        done = 0
        while done < n:
            k = min(per_launch, n - done)
            if k == 1:
                ctrl.step_plant_async(xp, up, 1)
            else:
                ctrl.run_closed_loop_async(xp, k, up)
            done += k

    def timed(n, per_launch):
        ctrl.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(n, per_launch)
        ctrl.sync()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / n

    run(args.warmup)
    run(min(args.warmup, 10), 1)
    ms_per_step = timed(args.steps, spl)
    ms_per_step_single = timed(args.steps, 1) if spl > 1 else ms_per_step
    rollout_steps = wl.K * wl.T
    value = rollout_steps / (ms_per_step / 1e3)

    # profiled pass of the same length: per-kernel HIP events on the library's stream
    ctrl.set_profiling(True)
    run(args.steps)
    times = ctrl.kernel_times()
    ctrl.set_profiling(False)
    roll_ms = times["rollout"][0]
    if wl.name == "quadrotor_mlp":
        ops = MLP_FLOP_PER_ROLLOUT_STEP * rollout_steps
        achieved = ops / (roll_ms / 1e3) / 1e12
        roofline = dict(bound="mfma", kernel="mlp_rollout", achieved=round(achieved, 3), peak=BF16_MFMA_PEAK_TFLOPS,
                        unit="TFLOP/s", frac=round(achieved / BF16_MFMA_PEAK_TFLOPS, 5), traffic=None,
                        alg_flop_per_launch=ops, kernel_ms=round(roll_ms, 5),
                        kernel_ms_all={k: round(v[0], 5) for k, v in times.items()},
                        launches_timed=times["rollout"][1],
                        mlp_train_seconds=round(wl.params["mlp"].train_seconds, 3),
                        mlp_final_loss=wl.params["mlp"].final_loss)
    else:
        ops = ALG_OPS_PER_ROLLOUT_STEP[wl.name] * rollout_steps
        achieved = ops / (roll_ms / 1e3) / 1e12
        roofline = dict(bound="alu", kernel="rollout", achieved=round(achieved, 4), peak=round(ALU_PEAK_TFLOPS, 2),
                        unit="TFLOP/s", frac=round(achieved / ALU_PEAK_TFLOPS, 5), traffic=measured_traffic(wl.name),
                        peak_published_fp32=PUBLISHED_FP32_TFLOPS,
                        alg_ops_per_launch=ops, kernel_ms=round(roll_ms, 5),
                        kernel_ms_all={k: round(v[0], 5) for k, v in times.items()},
                        launches_timed=times["rollout"][1])

    out = dict(metric=METRIC, value=round(value, 1), unit="rollout-steps/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(ms_per_step, 5), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload=f"{wl.name} K={wl.K} T={wl.T} nu={wl.nu} (1 iteration per control step"
                                    f"{', cost-to-go weighting' if ctg else ''})",
                           K=wl.K, T=wl.T, n=wl.n, m=wl.m, nu=wl.nu, lam=wl.lam, n_iters=1,
                           precision="FP32 rollouts, FP64 weights/normaliser/update", parallelism="single GPU"),
               mppi_iters_per_s=round(1e3 / ms_per_step, 1), roofline=roofline,
               launch=dict(steps_per_launch=spl, ms_per_step_one_launch_per_step=round(ms_per_step_single, 5),
                           rollout_steps_per_s_one_launch_per_step=round(rollout_steps / (ms_per_step_single / 1e3), 1)))
    if args.serving_seconds > 0:
        out["serving"] = serving_bench(args.serving_seconds, args.plain_seconds)
    # (the oracle leg runs path weighting: the cost-to-go parity is in the tests)
    if not args.no_cpu and wl.name != "quadrotor_mlp" and not ctg:
        # the CPU leg: the oracle timed on a bounded sample, and one more control step of the
        # timed controller checked against it from the same state, sequence and iteration
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
        out["cpu_baseline"]["value"] = round(out["cpu_baseline"]["value"], 1)
        if not args.no_parity:
            out["cpu_baseline"]["parity"] = parity_spot_check(wl, ctrl, x_dev.cpu().numpy())
    ctrl.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
