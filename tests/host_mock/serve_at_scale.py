"""Drive the serving runtime at the bench's scale (256 controllers of the serving mix) through
every batching mode, the pre-admitted replay and the session replay with a binding HBM budget.
Run in a child process against libmppi built with AddressSanitizer and linked to the HIP
stand-in (tests/host_mock/hip_mock.cpp); the kernels do not run, so only the host logic is
exercised.  Prints one line per leg."""
import sys

import numpy as np

sys.path.insert(0, sys.argv[1])
import paper_1509_01149_amd as P   # noqa: E402
import workloads as W              # noqa: E402
from bench import serving_mix_workloads, workspace_bytes   # noqa: E402

seconds = float(sys.argv[2])
wls = serving_mix_workloads(256)
need = np.array([workspace_bytes(w) for w in wls])
budget = int(0.75 * need.sum())
modes = dict(batched=P.SERVE_BATCHED, graph=P.SERVE_BATCHED_GRAPH, plain=P.SERVE_PLAIN)
trace = W.poisson_arrivals(256, 50.0, seconds)
for name, mode in modes.items():
    with P.Server(max_slots=256, max_inflight=3, max_batch=256, mode=mode, hbm_budget_bytes=budget) as srv:
        slots = []
        for c, wl in enumerate(wls):
            try:
                slots.append(srv.admit(**P.controller_args(wl)))
            except P.MppiError as e:
                assert e.code == P.binding.EBUSY
                slots.append(-1)
        slots = np.array(slots)
        ev = [(t, c) for t, c in trace if slots[c] >= 0]
        ci = np.array([c for _, c in ev])
        td, u0, st = srv.replay(np.array([t for t, _ in ev]), slots[ci], [np.pad(wls[c].x0, (0, 16 - wls[c].n)) for c in ci])
        assert len(td) == len(ev) and srv.stats()["requests_done"] == len(ev)
        print(f"{name}: replay of {len(ev)} requests, {int((slots >= 0).sum())} controllers admitted", flush=True)
    with P.Server(max_slots=256, max_inflight=3, max_batch=256, mode=mode, hbm_budget_bytes=budget) as srv:
        t_start, t_end = W.serving_sessions(256, start_s=seconds / 4, min_life_s=seconds / 3, max_life_s=seconds / 2)
        sess_trace = W.session_arrivals(t_start, t_end, 50.0)
        si = np.array([c for _, c in sess_trace])
        td, u0, st, ta, tr = srv.replay_sessions([P.controller_args(w) for w in wls], t_start, t_end,
                                                 np.array([t for t, _ in sess_trace]), si,
                                                 [np.pad(wls[c].x0, (0, 16 - wls[c].n)) for c in si])
        assert np.all(ta >= 0) and np.all(tr >= ta) and srv.stats()["bytes_used"] == 0
        print(f"{name}: sessions replay of {len(si)} requests, {int(np.sum(ta - t_start > 1e-3))} sessions queued",
              flush=True)
print("done", flush=True)
