"""Checks shared by the GPU solve-parity tests (single and batched): the
control gradient of every DAL iteration and the projected control step
Pi_E(eps - tau G) of Alg. 1, compared with the FP64 oracle."""
import numpy as np


def rel2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def grad_errors(got, ref):
    """Relative l2 error of the control gradient of every DAL iteration whose
    oracle gradient is not negligible (norm above 1e-6 of the largest one)."""
    norms = np.linalg.norm(ref.reshape(ref.shape[0], ref.shape[1], -1), axis=2)
    big = norms > 1e-6 * norms.max()
    return np.array([rel2(got[j, i], ref[j, i]) for j, i in zip(*np.nonzero(big))])


def own_step_errors(out, ref, eps_min=2.0, eps_max=1100.0):
    """Under control replay the GPU logs Pi_E(eps - tau G) from the replayed base
    controls, the replayed tau and its own gradient G.  Returns, per accepted
    step, (the difference from that formula evaluated here in FP64 on the
    GPU's logged gradient, the difference from the oracle's accepted controls,
    the bound tau |G_gpu - G_oracle|_inf that the 1-Lipschitz projection puts
    on the latter)."""
    dec = ref["decisions"]
    rows = []
    M, P = dec.shape
    base = None
    for j in range(M):
        for i in range(P):
            if dec[j, i] <= 0:
                continue
            if base is None:
                base = np.full_like(ref["eps_log"][j, i], 57.0)
            tau = dec[j, i]
            mine = np.clip(base - tau * out["grad_log"][j, i], eps_min, eps_max)
            e_formula = float(np.max(np.abs(out["eps_log"][j, i] - mine)))
            e_oracle = float(np.max(np.abs(out["eps_log"][j, i] - ref["eps_log"][j, i])))
            bound = float(tau * np.max(np.abs(out["grad_log"][j, i] - ref["grad_log"][j, i])))
            rows.append((e_formula, e_oracle, bound))
            base = ref["eps_log"][j, i]
    return np.array(rows)
