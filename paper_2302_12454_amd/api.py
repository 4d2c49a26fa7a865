"""Python binding of the SSQA C ABI (include/ssqa.h): argument marshalling only.

Every computation runs in libssqa.so: the sweep, the energies and the plane split
in HIP kernels on the GPU, the schedules and the GI mapping in the library's
host code.  PyTorch supplies device memory and the current HIP stream.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

from . import _lib

SSQA_NO_TARGET = -(2 ** 63)


class SSQAError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = _lib.load()
        name = lib.ssqa_status_string(status).decode()
        msg = lib.ssqa_last_error().decode()
        super().__init__(f"{where}: {name}: {msg}")
        self.status = status
        self.name = name


def _check(status: int, where: str) -> None:
    if status != 0:
        raise SSQAError(status, where)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class Problem:
    """An integer Ising model resident on one device (ssqa_create_problem)."""

    def __init__(self, h, J, device: int = 0):
        lib = _lib.load()
        h = _i32(h)
        J = _i32(J)
        n = int(h.shape[0])
        if J.shape != (n, n):
            raise ValueError(f"J must be {n} x {n}")
        handle = ctypes.c_void_p()
        _check(lib.ssqa_create_problem(n, _ptr(h, ctypes.c_int32), _ptr(J, ctypes.c_int32), int(device),
                                       ctypes.byref(handle)), "ssqa_create_problem")
        self._handle = handle
        self.device = int(device)
        self.n = n

    @property
    def handle(self):
        return self._handle

    @property
    def planes(self) -> int:
        return int(_lib.load().ssqa_problem_planes(self._handle))

    @property
    def padded(self) -> int:
        return int(_lib.load().ssqa_problem_padded(self._handle))

    @property
    def fp4_exact(self) -> bool:
        return bool(_lib.load().ssqa_problem_fp4_exact(self._handle))

    def close(self) -> None:
        if getattr(self, "_handle", None) is not None and self._handle.value:
            _lib.load().ssqa_destroy_problem(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ssqa_create_problem(h, J, device: int = 0) -> Problem:
    return Problem(h, J, device)


@dataclass
class AnnealState:
    """State of an anneal after ``cycle`` cycles (ssqa_anneal_state): counters int8 [T, R, N] and the
    delayed spins sigma(t - s), s = 1..d, bit-packed as int32 [T, R, d, ceil(N / 32)] (None when d = 0)."""
    counters: "object"
    history: "object | None"
    cycle: int


@dataclass
class AnnealResult:
    best_energy: "object"          # torch int64 [T] on the device
    first_hit: "object"            # torch int32 [T]
    energy_trace: "object | None"  # torch int32 [SC + 1, T, R]
    final_is: "object | None"      # torch int8 [T, R, N]
    checkpoint: "AnnealState | None" = None


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _alloc_outputs(problem: Problem, trials: int, replicas: int, cycles: int, trace: bool, final_is: bool):
    import torch
    dev = torch.device("cuda", problem.device)
    return AnnealResult(
        best_energy=torch.empty(trials, dtype=torch.int64, device=dev),
        first_hit=torch.empty(trials, dtype=torch.int32, device=dev),
        energy_trace=(torch.empty((cycles + 1, trials, replicas), dtype=torch.int32, device=dev) if trace else None),
        final_is=(torch.empty((trials, replicas, problem.n), dtype=torch.int8, device=dev) if final_is else None),
    )


def _params(*, replicas, trials, cycles, jperp, i0, alpha, noise_amp, delay, seed, coupling_mode=0, target=None,
            cycles_per_launch=0, block_columns=0, operand_format=0):
    jperp = _i32(jperp)
    i0 = _i32(i0)
    if len(jperp) < cycles or len(i0) < cycles:
        raise ValueError("schedules shorter than cycles")
    p = _lib.AnnealParams()
    p.replicas, p.trials, p.cycles = int(replicas), int(trials), int(cycles)
    p.delay, p.alpha, p.noise_amp = int(delay), int(alpha), int(noise_amp)
    p.coupling_mode, p.cycles_per_launch = int(coupling_mode), int(cycles_per_launch)
    p.jperp = _ptr(jperp, ctypes.c_int32)
    p.i0 = _ptr(i0, ctypes.c_int32)
    p.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    p.target_energy = SSQA_NO_TARGET if target is None else int(target)
    p.block_columns = int(block_columns)
    p.operand_format = int(operand_format)
    return p, (jperp, i0)          # keep the arrays alive as long as the struct


def _state_struct(state: "AnnealState | None"):
    if state is None:
        return None
    st = _lib.AnnealState()
    st.counters = state.counters.data_ptr()
    st.history = state.history.data_ptr() if state.history is not None else None
    return st


def _outputs(out: AnnealResult):
    o = _lib.AnnealOutputs()
    o.best_energy = out.best_energy.data_ptr()
    o.first_hit = out.first_hit.data_ptr()
    o.energy_trace = out.energy_trace.data_ptr() if out.energy_trace is not None else None
    o.final_is = out.final_is.data_ptr() if out.final_is is not None else None
    ck = _state_struct(out.checkpoint)
    if ck is not None:
        o.checkpoint = ctypes.pointer(ck)
    return o, ck


def ssqa_anneal(problem: Problem, *, replicas: int, trials: int, cycles: int, jperp, i0, alpha: int,
                noise_amp: int, delay: int, seed: int, coupling_mode: int = 0, target=None,
                trace: bool = False, final_is: bool = False, cycles_per_launch: int = 0, block_columns: int = 0,
                operand_format: int = 0, stream=None, out: AnnealResult | None = None,
                stop_cycle: int = 0, resume: "AnnealState | None" = None, checkpoint: bool = False,
                split_rows: int = 0) -> AnnealResult:
    """ssqa_anneal on torch-owned device outputs.  Asynchronous on ``stream`` (default: the
    current stream).  ``out`` may carry preallocated outputs of the right shapes.  ``split_rows`` picks
    the row-split form (0: automatic, -1: never, k > 0: from k padded rows on; see ssqa.h).

    Checkpoint / resume: ``checkpoint=True`` returns the state after the last cycle run (``stop_cycle``,
    or all ``cycles``) in ``result.checkpoint``; ``resume=state`` continues from it (pass the interrupted
    run's ``out`` as well, since best energies and first hits carry over)."""
    return _anneal_call("ssqa_anneal", **locals())


def ssqa_anneal_noalloc(problem: Problem, *, replicas: int, trials: int, cycles: int, jperp, i0, alpha: int,
                        noise_amp: int, delay: int, seed: int, coupling_mode: int = 0, target=None,
                        trace: bool = False, final_is: bool = False, cycles_per_launch: int = 0,
                        block_columns: int = 0, operand_format: int = 0, stream=None,
                        out: AnnealResult | None = None, stop_cycle: int = 0, resume: "AnnealState | None" = None,
                        checkpoint: bool = False, split_rows: int = 0) -> AnnealResult:
    """ssqa_anneal_noalloc: ssqa_anneal with the anneal's device state in the library's fixed per-device
    scratch (no device allocation by the library).  Same arguments and results as ``ssqa_anneal``; the
    outputs are still torch tensors unless ``out`` brings them."""
    return _anneal_call("ssqa_anneal_noalloc", **locals())


def _anneal_call(fn: str, *, problem, replicas, trials, cycles, jperp, i0, alpha, noise_amp, delay, seed,
                 coupling_mode, target, trace, final_is, cycles_per_launch, block_columns, operand_format,
                 stream, out, stop_cycle, resume, checkpoint, split_rows=0) -> AnnealResult:
    import torch
    lib = _lib.load()
    if out is None:
        out = _alloc_outputs(problem, trials, replicas, cycles, trace, final_is)
    if checkpoint:
        dev = out.best_energy.device
        words = (problem.n + 31) // 32
        out.checkpoint = AnnealState(
            counters=torch.empty((trials, replicas, problem.n), dtype=torch.int8, device=dev),
            history=(torch.empty((trials, replicas, delay, words), dtype=torch.int32, device=dev) if delay > 0
                     else None),
            cycle=stop_cycle if stop_cycle else cycles)
    p, keep = _params(replicas=replicas, trials=trials, cycles=cycles, jperp=jperp, i0=i0, alpha=alpha,
                      noise_amp=noise_amp, delay=delay, seed=seed, coupling_mode=coupling_mode, target=target,
                      cycles_per_launch=cycles_per_launch, block_columns=block_columns,
                      operand_format=operand_format)
    p.stop_cycle = int(stop_cycle)
    p.split_rows = int(split_rows)
    rs = _state_struct(resume)
    if resume is not None:
        p.start_cycle = int(resume.cycle)
        p.resume = ctypes.pointer(rs)
    o, ck = _outputs(out)
    _check(getattr(lib, fn)(problem.handle, ctypes.byref(p), ctypes.byref(o), _stream_handle(stream)), fn)
    del keep, rs, ck
    return out


class Batch:
    """ssqa_batch_create / run / destroy: many anneals in one persistent launch replayed from a HIP graph.

    ``jobs`` is a list of (problem, kwargs) where kwargs are ssqa_anneal's keyword arguments (replicas,
    trials, cycles, jperp, i0, alpha, noise_amp, delay, seed, coupling_mode, target, trace, final_is).
    """

    def __init__(self, jobs):
        lib = _lib.load()
        n = len(jobs)
        self.problems = [p for p, _ in jobs]
        self.results = []
        self._keep = []
        params = (_lib.AnnealParams * n)()
        outs = (_lib.AnnealOutputs * n)()
        handles = (ctypes.c_void_p * n)()
        for i, (prob, kw) in enumerate(jobs):
            kw = dict(kw)
            trace = kw.pop("trace", False)
            final_is = kw.pop("final_is", False)
            res = _alloc_outputs(prob, kw["trials"], kw["replicas"], kw["cycles"], trace, final_is)
            p, keep = _params(**kw)
            params[i] = p
            outs[i] = _outputs(res)[0]
            handles[i] = prob.handle
            self.results.append(res)
            self._keep.append(keep)
        handle = ctypes.c_void_p()
        _check(lib.ssqa_batch_create(n, handles, params, outs, ctypes.byref(handle)), "ssqa_batch_create")
        self._handle = handle

    @property
    def blocks(self) -> int:
        return int(_lib.load().ssqa_batch_blocks(self._handle))

    def run(self, stream=None):
        _check(_lib.load().ssqa_batch_run(self._handle, _stream_handle(stream)), "ssqa_batch_run")
        return self.results

    def close(self):
        if getattr(self, "_handle", None) is not None and self._handle.value:
            _lib.load().ssqa_batch_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ssqa_batch_create(jobs) -> Batch:
    return Batch(jobs)


def _tile_dict(t) -> dict:
    return {"block_columns": int(t.block_columns), "trials_per_block": int(t.trials_per_block),
            "operands": "fp4" if t.operand_format == 2 else "int8", "blocks": int(t.blocks),
            "ms_per_cycle": float(t.ms_per_cycle)}


def _anneal_params_only(kw: dict):
    kw = dict(kw)
    for key in ("trace", "final_is", "stream", "out", "stop_cycle", "resume", "checkpoint"):
        kw.pop(key, None)
    return _params(**kw)


def ssqa_tune_anneal(problem: Problem, *, probe_cycles: int = 20, stream=None, **anneal):
    """ssqa_tune_anneal: time every legal tiling of this anneal (ssqa_anneal's keyword arguments, with
    block_columns and operand_format left automatic) on its first ``probe_cycles`` cycles and record the
    fastest.  Returns (chosen, candidates) as dicts."""
    lib = _lib.load()
    p, keep = _anneal_params_only(anneal)
    cap = 64
    cands = (_lib.Tile * cap)()
    count = ctypes.c_int32()
    chosen = _lib.Tile()
    _check(lib.ssqa_tune_anneal(problem.handle, ctypes.byref(p), int(probe_cycles), _stream_handle(stream), cands, cap,
                                ctypes.byref(count), ctypes.byref(chosen)), "ssqa_tune_anneal")
    del keep
    return _tile_dict(chosen), [_tile_dict(cands[i]) for i in range(min(count.value, cap))]


def ssqa_tune_batch(jobs, *, probe_cycles: int = 20, stream=None) -> dict:
    """ssqa_tune_batch over (problem, kwargs) jobs as for Batch: the fastest 128-column floor (0 = never)."""
    lib = _lib.load()
    n = len(jobs)
    params = (_lib.AnnealParams * n)()
    handles = (ctypes.c_void_p * n)()
    keep = []
    for i, (prob, kw) in enumerate(jobs):
        p, k = _anneal_params_only(kw)
        params[i] = p
        handles[i] = prob.handle
        keep.append(k)
    rows = ctypes.c_int32()
    ms = ctypes.c_double()
    _check(lib.ssqa_tune_batch(n, handles, params, int(probe_cycles), _stream_handle(stream), ctypes.byref(rows),
                               ctypes.byref(ms)), "ssqa_tune_batch")
    del keep
    return {"wide_rows": int(rows.value), "ms_per_cycle": float(ms.value)}


def ssqa_tune_lookup(problem: Problem, **anneal):
    """The tiling ssqa_anneal would take for these arguments, and whether the tuner's cache chose it."""
    lib = _lib.load()
    p, keep = _anneal_params_only(anneal)
    t = _lib.Tile()
    tuned = ctypes.c_int32()
    _check(lib.ssqa_tune_lookup(problem.handle, ctypes.byref(p), ctypes.byref(t), ctypes.byref(tuned)),
           "ssqa_tune_lookup")
    del keep
    return _tile_dict(t), bool(tuned.value)


def ssqa_tune_set(problem: Problem, tile: dict, **anneal) -> None:
    """Record ``tile`` (block_columns, trials_per_block, operands) for the shape of these anneal arguments."""
    lib = _lib.load()
    p, keep = _anneal_params_only(anneal)
    t = _lib.Tile(int(tile["block_columns"]), int(tile["trials_per_block"]),
                  2 if tile.get("operands", "int8") == "fp4" else 1, 0, float(tile.get("ms_per_cycle", 0.0)))
    _check(lib.ssqa_tune_set(problem.handle, ctypes.byref(p), ctypes.byref(t)), "ssqa_tune_set")
    del keep


def ssqa_tune_save(path: str) -> None:
    _check(_lib.load().ssqa_tune_save(os.fsencode(path)), "ssqa_tune_save")


def ssqa_tune_load(path: str) -> int:
    n = ctypes.c_int32()
    _check(_lib.load().ssqa_tune_load(os.fsencode(path), ctypes.byref(n)), "ssqa_tune_load")
    return int(n.value)


def ssqa_tune_entries() -> int:
    return int(_lib.load().ssqa_tune_entries())


def ssqa_tune_clear() -> None:
    _lib.load().ssqa_tune_clear()


def ssqa_energy(problem: Problem, spins, stream=None):
    """H_p of each row of ``spins`` (torch int8 [cols, N] of +-1 on the device) -> int64 [cols]."""
    import torch
    lib = _lib.load()
    spins = spins.contiguous()
    if spins.dtype != torch.int8 or spins.dim() != 2 or spins.shape[1] != problem.n:
        raise ValueError("spins must be int8 [cols, N]")
    cols = int(spins.shape[0])
    energies = torch.empty(cols, dtype=torch.int64, device=spins.device)
    _check(lib.ssqa_energy(problem.handle, ctypes.c_void_p(spins.data_ptr()), cols,
                           ctypes.c_void_p(energies.data_ptr()), _stream_handle(stream)), "ssqa_energy")
    return energies


def ssqa_qmc_energy(problem: Problem, counters, jperp: int, stream=None):
    """QMC Hamiltonian (Eq. 4) per trial from counters (torch int8 [T, R, N] on the device) -> int64 [T]."""
    import torch
    lib = _lib.load()
    counters = counters.contiguous()
    if counters.dtype != torch.int8 or counters.dim() != 3 or counters.shape[2] != problem.n:
        raise ValueError("counters must be int8 [T, R, N]")
    T, R = int(counters.shape[0]), int(counters.shape[1])
    energies = torch.empty(T, dtype=torch.int64, device=counters.device)
    _check(lib.ssqa_qmc_energy(problem.handle, ctypes.c_void_p(counters.data_ptr()), T, R, int(jperp),
                               ctypes.c_void_p(energies.data_ptr()), _stream_handle(stream)), "ssqa_qmc_energy")
    return energies


@dataclass
class SAResult:
    best_energy: object            # torch int64 [T]
    first_hit: object              # torch int32 [T]
    final_energy: object = None    # torch int64 [T]
    final_spins: object = None     # torch int8 [T, N]
    energy_trace: object = None    # torch int64 [cycles + 1, T]


def ssqa_sa_anneal(problem: Problem, *, trials: int, beta, seed: int = 0, target=None, final_state: bool = True,
                   trace: bool = False, stream=None) -> SAResult:
    """Serial single-spin Metropolis chains (the SA baseline of Section 4.4) on the problem's device;
    ``beta`` is the per-cycle inverse temperature at the problem's integer scale."""
    import torch
    lib = _lib.load()
    beta = np.ascontiguousarray(np.asarray(beta, dtype=np.float64))
    cycles = int(beta.shape[0])
    dev = torch.device("cuda", problem.device)
    res = SAResult(best_energy=torch.empty(trials, dtype=torch.int64, device=dev),
                   first_hit=torch.empty(trials, dtype=torch.int32, device=dev))
    if final_state:
        res.final_energy = torch.empty(trials, dtype=torch.int64, device=dev)
        res.final_spins = torch.empty((trials, problem.n), dtype=torch.int8, device=dev)
    if trace:
        res.energy_trace = torch.empty((cycles + 1, trials), dtype=torch.int64, device=dev)
    p = _lib.SAParams()
    p.trials = int(trials)
    p.cycles = cycles
    p.beta = _ptr(beta, ctypes.c_double)
    p.seed = int(seed) & (2 ** 64 - 1)
    p.target_energy = SSQA_NO_TARGET if target is None else int(target)
    o = _lib.SAOutputs()

    def ptr(t):
        return None if t is None else t.data_ptr()

    o.best_energy, o.first_hit = ptr(res.best_energy), ptr(res.first_hit)
    o.final_energy, o.final_spins, o.energy_trace = ptr(res.final_energy), ptr(res.final_spins), ptr(res.energy_trace)
    _check(lib.ssqa_sa_anneal(problem.handle, ctypes.byref(p), ctypes.byref(o), _stream_handle(stream)),
           "ssqa_sa_anneal")
    return res


def ssqa_sa_schedule(cycles: int, t_start: float = 1000.0, t_end: float = 0.1, scale: int = 12) -> np.ndarray:
    out = np.zeros(max(cycles, 1), dtype=np.float64)
    _check(_lib.load().ssqa_sa_schedule(cycles, float(t_start), float(t_end), scale, _ptr(out, ctypes.c_double)),
           "ssqa_sa_schedule")
    return out[:cycles]


def ssqa_sa_accept_threshold(de: int, beta: float) -> float:
    return float(_lib.load().ssqa_sa_accept_threshold(int(de), float(beta)))


def ssqa_jperp_schedule(cycles: int, tau: int, beta: int, jmin_num: int, jmax_num: int, den: int,
                        scale: int) -> np.ndarray:
    out = np.zeros(max(cycles, 1), dtype=np.int32)
    _check(_lib.load().ssqa_jperp_schedule(cycles, tau, beta, jmin_num, jmax_num, den, scale,
                                           _ptr(out, ctypes.c_int32)), "ssqa_jperp_schedule")
    return out[:cycles]


def ssqa_ssa_i0_schedule(cycles: int, tau: int, growth: int, i0_min: int, i0_max: int, scale: int) -> np.ndarray:
    out = np.zeros(max(cycles, 1), dtype=np.int32)
    _check(_lib.load().ssqa_ssa_i0_schedule(cycles, tau, growth, i0_min, i0_max, scale,
                                            _ptr(out, ctypes.c_int32)), "ssqa_ssa_i0_schedule")
    return out[:cycles]


def ssqa_gi_to_ising(a1, a2, c1: int = 1, c2: int = 1, scale: int = 12):
    """GI pair -> (h int32 [N], J int32 [N, N], E* int) computed by the library."""
    a1 = np.ascontiguousarray(np.asarray(a1, dtype=np.uint8))
    a2 = np.ascontiguousarray(np.asarray(a2, dtype=np.uint8))
    n = a1.shape[0]
    N = n * n
    h = np.zeros(N, dtype=np.int32)
    J = np.zeros((N, N), dtype=np.int32)
    e = ctypes.c_int64()
    _check(_lib.load().ssqa_gi_to_ising(n, _ptr(a1, ctypes.c_uint8), _ptr(a2, ctypes.c_uint8), c1, c2, scale,
                                        _ptr(h, ctypes.c_int32), _ptr(J, ctypes.c_int32), ctypes.byref(e)),
           "ssqa_gi_to_ising")
    return h, J, int(e.value)


def ssqa_philox4x32_10(ctr, key) -> list[int]:
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    _lib.load().ssqa_philox4x32_10(c, k, o)
    return [int(x) for x in o]


REQUEST_STATES = {0: "queued", 1: "running", 2: "done", 3: "cancelled", 4: "failed"}


class Server:
    """ssqa_server_*: continuous batching of anneal requests with memory-based admission."""

    def __init__(self, device: int = 0, cycles_per_step: int = 100, max_active: int = 64,
                 memory_budget: int = 64 << 30, split_rows: int = 0):
        lib = _lib.load()
        cfg = _lib.ServerConfig(int(device), int(cycles_per_step), int(max_active), int(memory_budget),
                                int(split_rows))
        handle = ctypes.c_void_p()
        _check(lib.ssqa_server_create(ctypes.byref(cfg), ctypes.byref(handle)), "ssqa_server_create")
        self._handle = handle
        self._trials = {}

    def submit(self, h, J, *, early_exit: bool = False, **anneal) -> int:
        """Queue a request; ``anneal`` takes ssqa_anneal's parameters (replicas, trials, cycles, jperp, i0,
        alpha, noise_amp, delay, seed, coupling_mode, target, block_columns)."""
        lib = _lib.load()
        h = _i32(h)
        J = _i32(J)
        n = int(h.shape[0])
        if J.shape != (n, n):
            raise ValueError(f"J must be {n} x {n}")
        p, keep = _params(**anneal)
        req = _lib.Request()
        req.n_spins = n
        req.h = _ptr(h, ctypes.c_int32)
        req.J = _ptr(J, ctypes.c_int32)
        req.params = p
        req.early_exit = 1 if early_exit else 0
        rid = ctypes.c_int64()
        _check(lib.ssqa_server_submit(self._handle, ctypes.byref(req), ctypes.byref(rid)), "ssqa_server_submit")
        del keep
        self._trials[int(rid.value)] = int(anneal["trials"])
        return int(rid.value)

    def step(self, stream=None) -> int:
        active = ctypes.c_int32()
        _check(_lib.load().ssqa_server_step(self._handle, _stream_handle(stream), ctypes.byref(active)),
               "ssqa_server_step")
        return int(active.value)

    def poll(self, rid: int) -> dict:
        T = self._trials[rid]
        info = _lib.RequestInfo()
        best = np.zeros(T, dtype=np.int64)
        hit = np.zeros(T, dtype=np.int32)
        _check(_lib.load().ssqa_server_poll(self._handle, rid, ctypes.byref(info), _ptr(best, ctypes.c_int64),
                                            _ptr(hit, ctypes.c_int32)), "ssqa_server_poll")
        return {"state": REQUEST_STATES.get(info.state, str(info.state)), "status": int(info.status),
                "cycles_done": int(info.cycles_done), "submit_s": info.submit_s, "admit_s": info.admit_s,
                "done_s": info.done_s, "memory_bytes": int(info.memory_bytes), "best": best, "first_hit": hit}

    def cancel(self, rid: int) -> None:
        _check(_lib.load().ssqa_server_cancel(self._handle, rid), "ssqa_server_cancel")

    def stats(self) -> dict:
        st = _lib.ServerStats()
        _check(_lib.load().ssqa_server_stats(self._handle, ctypes.byref(st)), "ssqa_server_stats")
        return {"queued": st.queued, "active": st.active, "memory_in_use": int(st.memory_in_use),
                "spin_updates": st.spin_updates, "elapsed_s": st.elapsed_s}

    def close(self) -> None:
        if getattr(self, "_handle", None) is not None and self._handle.value:
            _lib.load().ssqa_server_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ssqa_server_create(**kw) -> Server:
    return Server(**kw)
