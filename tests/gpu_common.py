"""Helpers shared by the GPU parity tests (inputs, comparisons and the support rule)."""
import json
import os

import numpy as np
import scipy.sparse as sp


def max_abs_diff(a: sp.spmatrix, b: sp.spmatrix) -> float:
    d = (sp.csr_matrix(a) - sp.csr_matrix(b))
    return float(np.abs(d.data).max()) if d.nnz else 0.0


def support_mismatch(gpu: sp.spmatrix, ref: sp.spmatrix):
    """Entries in the support of exactly one of the two matrices."""
    g = sp.csr_matrix(gpu).copy()
    r = sp.csr_matrix(ref).copy()
    g.data[:] = 1.0
    r.data[:] = 1.0
    d = (g - r).tocoo()
    keep = d.data != 0
    return list(zip(d.row[keep].tolist(), d.col[keep].tolist()))


def _report(rec: dict) -> None:
    """Print a support record and append it to $CONCORD_TEST_REPORT (JSON lines) if set."""
    print("[support]", json.dumps(rec), flush=True)
    path = os.environ.get("CONCORD_TEST_REPORT")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps(rec) + "\n")


def check_support(label, precision, lam1, tau, got_next, want_next, gpu_prev, want_prev,
                  gpu_cands, oracle_grad_at):
    """Support rule of the parity tests for one step Omega^k -> Omega^{k+1}.

    An entry may be in the support of exactly one of the two iterates only when the
    oracle's prox argument u = (omega^k_ij - tau G_ij) / tau lies near the threshold:
    its margin | |u_ij| - lam1 | / lam1 must be
      FP64:          at most 1e-6 (the band of the method's tolerances);
      FP32, BF16x3:  at most the step's measured error of u on the GPU side,
                     (max_A |G_gpu - G_oracle| + max |Omega^k_gpu - Omega^k_oracle| / tau) / lam1,
                     with the gradient error measured over the GPU's candidate set A.
    Every mismatch is reported with its margin.

    gpu_cands: (omega, grad) CSR matrices of the GPU step's candidate set (at the GPU's
    Omega^k); oracle_grad_at(entries) -> the oracle's G at Omega^k_oracle for those entries.
    Returns the measured error bound (in units of lam1) for reduced precision, else 0.
    """
    mism = support_mismatch(got_next, want_next)
    want_prev = sp.csr_matrix(want_prev)
    bound = 0.0
    if precision != "fp64":
        _, ggpu = gpu_cands
        coo = ggpu.tocoo()
        entries = list(zip(coo.row.tolist(), coo.col.tolist()))
        g_or = np.asarray(oracle_grad_at(entries), dtype=np.float64)
        gerr = float(np.abs(coo.data - g_or).max()) if len(entries) else 0.0
        oerr = max_abs_diff(gpu_prev, want_prev)
        bound = (gerr + oerr / tau) / lam1
        _report({"case": label, "precision": precision, "grad_err": gerr, "omega_err": oerr,
                 "bound_over_lam1": bound, "mismatches": len(mism)})
    if not mism:
        return bound
    g_m = np.asarray(oracle_grad_at(mism), dtype=np.float64)
    for (i, j), g in zip(mism, g_m):
        u = (want_prev[i, j] - tau * g) / tau
        margin = abs(abs(u) - lam1) / lam1
        rec = {"case": label, "precision": precision, "i": int(i), "j": int(j),
               "margin_over_lam1": margin, "in_gpu": bool(sp.csr_matrix(got_next)[i, j] != 0)}
        _report(rec)
        if precision == "fp64":
            assert margin <= 1e-6, rec
        else:
            assert margin <= bound, (rec, bound)
    return bound


def oracle_grad_fn(omega_prev, X, lam2, variant="obs", S=None):
    """G of the oracle at omega_prev on listed entries: one by one from Y = Omega X^T
    (oracle.smooth_value_and_sampled_grads), or from S for a Cov problem without X."""
    from oracle import concord as oc

    def at(entries):
        entries = list(entries)
        if not entries:
            return np.zeros(0)
        if X is not None:
            _, G, _ = oc.smooth_value_and_sampled_grads(omega_prev, X, lam2, entries, [])
            return G
        W = np.asarray(sp.csr_matrix(omega_prev) @ S)
        G = oc.gradient(W, sp.csr_matrix(omega_prev), lam2)
        return np.array([G[i, j] for i, j in entries])
    return at
