"""Autotuner for the pair-kernel launch: picks the kernel variant, cluster size, cell
divisions, work items per cluster, schedule and residency for a given batch of
systems by timing candidates through the C ABI on the caller's own data.

A candidate is accepted only if its forces agree with the library defaults' forces
(they compute the same sums in another order or grouping, so they must agree to
rounding);
among the accepted candidates the one with the lowest median time per evaluation
(nb_build_cells + nb_nonbonded_forces with energy and virial) wins.  The search is
staged rather than exhaustive: kernel and cluster size first, then the cell
divisions, then items per cluster with the schedule and residency, each stage
starting from the best so far.

Choices are cached as JSON, keyed by a signature of the workload (system count,
atom count, mean density, cutoff, Ewald beta, precision, type count, device), in
the file named by NBHIP_TUNE_CACHE or ~/.cache/nbhip/tune.json.
"""

from __future__ import annotations

import hashlib
import json
import math
import os
import time
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import nbhip as H

CACHE_ENV = "NBHIP_TUNE_CACHE"
PARAM_KEYS = ("kernel", "cluster_size", "cell_div_xy", "cell_div_z", "split", "schedule", "wg_per_cu")


def cache_path() -> str:
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache", "nbhip", "tune.json")


def signature(batch, cutoff: float, beta: float, precision: int, device_name: str = "") -> str:
    """Workload key: what the best launch depends on (sizes to about 10 %, density to 1 %)."""
    n = int(batch.n_atoms)
    B = int(batch.n_systems)
    vol = float(np.prod(np.asarray(batch.box, dtype=np.float64).reshape(-1, 3), axis=1).sum())
    rho = n / vol if vol > 0 else 0.0
    key = {
        "B": B,
        "logN": round(math.log(max(n, 1)) / math.log(1.1)),
        "rho": round(rho, 3),
        "cutoff": round(float(cutoff), 4),
        "beta": round(float(beta), 4),
        "precision": int(precision),
        "T": int(batch.sigma.shape[0]),
        "device": device_name,
    }
    return hashlib.sha1(json.dumps(key, sort_keys=True).encode()).hexdigest()[:16] + ":" + json.dumps(key, sort_keys=True)


def load_cache(path: Optional[str] = None) -> Dict[str, dict]:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store_cache(key: str, entry: dict, path: Optional[str] = None) -> None:
    path = path or cache_path()
    data = load_cache(path)
    data[key] = entry
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def params_from(entry: dict, cutoff: float, beta: float, precision: int) -> "H.nb_params":
    return H.make_params(cutoff, beta, precision, **{k: int(entry.get(k, 0)) for k in PARAM_KEYS})


def stage_candidates(stage: int, best: dict, precision: int) -> List[dict]:
    """Candidates of one stage, as overrides of the best choice so far."""
    if stage == 0:
        out = [dict(kernel=H.NB_KERNEL_CLUSTER, cluster_size=8), dict(kernel=H.NB_KERNEL_CLUSTER, cluster_size=4),
               dict(kernel=H.NB_KERNEL_CLUSTER_HALF, cluster_size=8),
               dict(kernel=H.NB_KERNEL_CLUSTER_HALF, cluster_size=4)]
        return out
    if stage == 1:
        return [dict(cell_div_xy=xy, cell_div_z=z) for xy, z in ((2, 8), (2, 4), (2, 12), (1, 8), (3, 12))]
    if stage == 2:
        return [dict(split=s, schedule=sch, wg_per_cu=w) for s, sch, w in
                ((1, H.NB_SCHED_STATIC, 0), (2, H.NB_SCHED_STATIC, 0), (3, H.NB_SCHED_STATIC, 0),
                 (2, H.NB_SCHED_DYNAMIC, 12), (1, H.NB_SCHED_DYNAMIC, 16))]
    return []


def _time_config(batch, params, reps: int, warmup: int):
    """Median seconds per build + forces (energy and virial) and the forces."""
    import torch
    ws = H.alloc_workspace(batch, params)
    B = batch.n_systems
    force = torch.empty((batch.n_atoms, 3), dtype=torch.float64, device=batch.pos.device)
    energy = torch.empty(B, dtype=torch.float64, device=batch.pos.device)
    vir = torch.empty((B, 3, 3), dtype=torch.float64, device=batch.pos.device)

    def step():
        H.build_cells(batch, params, ws)
        H.nonbonded_forces(batch, params, ws, force, energy, vir)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for k in range(reps):
        step()
        ev[k + 1].record()
    torch.cuda.synchronize()
    times = [ev[k].elapsed_time(ev[k + 1]) * 1e-3 for k in range(reps)]
    status = H.read_status(ws)
    return float(np.median(times)), force.cpu().numpy(), status


def _rel(a, b) -> float:
    den = float(np.sqrt(np.mean(b * b)))
    return float(np.sqrt(np.mean((a - b) ** 2)) / den) if den > 0 else float(np.abs(a - b).max())


def tune(batch, cutoff: float, beta: float, precision: int, reps: int = 10, warmup: int = 3,
         budget_s: float = 60.0, use_cache: bool = True, verbose: bool = False) -> Tuple["H.nb_params", dict]:
    """Best launch parameters for this batch (and the record of the search)."""
    import torch
    dev = torch.cuda.get_device_name(batch.pos.device) if torch.cuda.is_available() else ""
    key = signature(batch, cutoff, beta, precision, dev)
    if use_cache:
        hit = load_cache().get(key)
        if hit is not None:
            return params_from(hit["params"], cutoff, beta, precision), dict(hit, cached=True)
    tol = 1e-12 if precision == H.NB_FP64 else 1e-5
    t_start = time.perf_counter()
    base = {k: 0 for k in PARAM_KEYS}
    t0, f_ref, st = _time_config(batch, params_from(base, cutoff, beta, precision), reps, warmup)
    tried = [dict(params=dict(base), sec=t0, accepted=st == 0)]
    best, best_t = dict(base), t0
    for stage in range(3):
        stage_best, stage_t = dict(best), best_t
        for over in stage_candidates(stage, best, precision):
            if time.perf_counter() - t_start > budget_s:
                break
            cand = dict(best, **over)
            if any(cand == t["params"] for t in tried):
                continue
            try:
                t, f, st = _time_config(batch, params_from(cand, cutoff, beta, precision), reps, warmup)
            except H.NbError as e:  # a choice the library rejects for this batch
                tried.append(dict(params=cand, error=str(e)))
                continue
            ok = st == 0 and _rel(f, f_ref) <= tol
            tried.append(dict(params=cand, sec=t, accepted=ok))
            if verbose:
                print(f"[tune] {cand} {t * 1e6:.1f} us {'ok' if ok else 'REJECTED'}", flush=True)
            if ok and t < stage_t:
                stage_best, stage_t = cand, t
        best, best_t = stage_best, stage_t
    entry = dict(params=best, sec=best_t, default_sec=t0, tried=tried, key=key,
                 search_s=time.perf_counter() - t_start)
    if use_cache:
        store_cache(key, entry)
    return params_from(best, cutoff, beta, precision), entry
