"""Helpers shared by the GPU parity tests: run the HIP library and the oracle on the
same seeded inputs and compare element by element (everything is integer, so the
bar is bit-exact equality)."""

from __future__ import annotations

from fractions import Fraction

import numpy as np

from oracle import gi, ssqa
from synth import random_gi_pair


def paper_schedules(cycles: int, tau: int = 100, scale: int = 12):
    """Table 2 defaults at scale S: J_perp 0 -> 1/2 in beta = 3 steps, I_0 = 2, n_rnd = 1."""
    q = ssqa.scaled(ssqa.jperp_schedule(cycles, tau, 3, 0, Fraction(1, 2)), scale)
    i0 = np.full(cycles, 2 * scale, dtype=np.int64)
    return q, i0, scale  # noise amplitude n_rnd * S = S


def gi_case(n: int, graph_seed: int, scale: int = 12):
    pair = random_gi_pair(n, 0.5, graph_seed)
    h, J, e_star = gi.gi_ising(pair.a1, pair.a2, scale)
    return h, J, e_star


def run_gpu(prob, *, replicas, trials, cycles, q, i0, alpha, noise, delay, seed, mode=0, target=None,
            cycles_per_launch=0, trace=True, final_is=True, block_columns=0, operand_format=0, split_rows=0):
    import torch
    import paper_2302_12454_amd as lib
    res = lib.ssqa_anneal(prob, replicas=replicas, trials=trials, cycles=cycles, jperp=q, i0=i0, alpha=alpha,
                          noise_amp=noise, delay=delay, seed=seed, coupling_mode=mode, target=target,
                          trace=trace, final_is=final_is, cycles_per_launch=cycles_per_launch,
                          block_columns=block_columns, operand_format=operand_format, split_rows=split_rows)
    torch.cuda.synchronize()
    return {
        "best": res.best_energy.cpu().numpy(),
        "first_hit": res.first_hit.cpu().numpy(),
        "trace": res.energy_trace.cpu().numpy() if trace else None,
        "Is": res.final_is.cpu().numpy() if final_is else None,
    }


def run_oracle(h, J, *, replicas, trials, cycles, q, i0, alpha, noise, delay, seed, mode=0, target=None):
    return ssqa.anneal(h, J, replicas, trials, cycles, q, i0, alpha, noise, delay, seed, coupling_mode=mode,
                       target=target)


def assert_same(gpu, ref, trial_idx=None, check_trace=True, check_is=True):
    """Bit-exact comparison of a GPU run with an oracle run (optionally on a subset of trials)."""
    sel = slice(None) if trial_idx is None else np.asarray(trial_idx)
    if check_trace:
        g = gpu["trace"][:, sel, :]
        assert g.shape == ref.energy.shape, (g.shape, ref.energy.shape)
        if not np.array_equal(g, ref.energy):
            bad = np.argwhere(g != ref.energy)
            t, b, k = bad[0]
            raise AssertionError(f"energy trace differs at {len(bad)} entries; first t={t} b={b} k={k}: "
                                 f"gpu {g[t, b, k]} oracle {ref.energy[t, b, k]}")
    assert np.array_equal(gpu["best"][sel], ref.best), (gpu["best"][sel], ref.best)
    assert np.array_equal(gpu["first_hit"][sel], ref.first_hit), (gpu["first_hit"][sel], ref.first_hit)
    if check_is:
        g = gpu["Is"][sel]
        if not np.array_equal(g, ref.Is):
            bad = np.argwhere(g != ref.Is)
            raise AssertionError(f"final Is differs at {len(bad)} entries, first {bad[0].tolist()}")
