"""Parity rules between the GPU path and the FP64 oracle (test infrastructure).

Distance rule (float32 path): for every returned pair,
    |d_gpu - d*| <= tol * max(d*, floor * (N*_i + N*_j))
where d* is the oracle distance and N* the oracle patch norms; the floor scales with the
operands of the cancellation N_i + N_j - 2C in Lemma 2 (exact zero distances are compared
against that scale rather than against zero).

Set rule: with t the oracle's K-th distance and tau = tol * max(t, floor*(N*_i + N*_jK)),
the GPU set holds min(K, |Cand|) distinct in-window candidates, every member has
d* <= t + tau, and every candidate with d* < t - tau is a member.  When the oracle's K-th
and (K+1)-th distances differ by more than tau this forces the exact oracle set.
"""
from __future__ import annotations

import numpy as np

from oracle import bm_oracle as O


class ParityReport:
    def __init__(self):
        self.rel = []
        self.strict_mismatch = 0
        self.tolerant_mismatch = 0
        self.order_violations = 0
        self.n_refs = 0
        self.messages = []

    def summary(self):
        r = np.concatenate(self.rel) if self.rel else np.zeros(1)
        return {"refs": self.n_refs, "rel_max": float(r.max()), "rel_p99": float(np.quantile(r, 0.99)),
                "rel_median": float(np.median(r)), "strict_set_mismatch": self.strict_mismatch,
                "tolerant_set_mismatch": self.tolerant_mismatch, "order_violations": self.order_violations}


def _check_row(rep, i, d, j, K, gi, gd, ni, norm_of, tol, floor):
    """One GPU row against the oracle's in-window distances d (indices j) of reference i;
    ni is the reference's oracle norm, norm_of(j) a candidate's."""
    ncand = d.size
    oidx, odist = O.select_k(d, j, K)
    lookup = dict(zip(j.tolist(), d.tolist()))
    rep.n_refs += 1
    kk = min(K, ncand)
    # padding
    if np.any(gi[kk:] != -1) or np.any(np.isfinite(gd[kk:])):
        rep.tolerant_mismatch += 1
        rep.messages.append(f"ref {i}: bad padding")
        return
    members = gi[:kk].tolist()
    if len(set(members)) != kk or any(m not in lookup for m in members):
        rep.tolerant_mismatch += 1
        rep.messages.append(f"ref {i}: non-candidate or duplicate indices {members}")
        return
    dstar = np.array([lookup[m] for m in members])
    nj = np.array([norm_of(m) for m in members])
    rel = np.abs(gd[:kk].astype(np.float64) - dstar) / np.maximum(dstar, floor * (ni + nj))
    rep.rel.append(rel)
    if np.any(rel > tol):
        rep.tolerant_mismatch += 1
        rep.messages.append(f"ref {i}: rel error {rel.max():.3e}")
    # ascending order of the GPU's own keys
    keys = list(zip(gd[:kk].tolist(), members))
    if keys != sorted(keys):
        rep.order_violations += 1
    # set rule
    t = odist[kk - 1]
    jk = int(oidx[kk - 1])
    tau = tol * max(t, floor * (ni + norm_of(jk)))
    if set(members) != set(oidx[:kk].tolist()):
        rep.strict_mismatch += 1
        must = {int(a) for a, b in zip(j, d) if b < t - tau}
        if np.any(dstar > t + tau) or not must.issubset(set(members)):
            rep.tolerant_mismatch += 1
            rep.messages.append(f"ref {i}: set rule violated")


def check(x, P, s, Wn, K, gpu_idx, gpu_dist, refs=None, tol=1e-4, floor=1e-2, report=None):
    """Check GPU rows (for reference numbers ``refs``, default all) against the oracle."""
    x64 = np.asarray(x, dtype=np.float64)
    if x64.ndim == 2:
        x64 = x64[None]
    C, H, W = x64.shape
    N = O.patch_norms(x64, P)
    rl = O.ref_list(H, W, P, s)
    sel = np.arange(len(rl)) if refs is None else np.asarray(refs)
    gpu_idx = np.asarray(gpu_idx)
    gpu_dist = np.asarray(gpu_dist)
    rep = report or ParityReport()
    for row, i in enumerate(sel):
        ry, rx = int(rl[i, 0]), int(rl[i, 1])
        d, j = O.window_distances(x64, P, Wn, ry, rx)
        _check_row(rep, i, d, j, K, gpu_idx[row], gpu_dist[row], N[ry, rx],
                   lambda m: N[m // W, m % W], tol, floor)
    return rep


def check3d(v, P, d, s, Wn, c, K, gpu_idx, gpu_dist, refs=None, tol=1e-4, floor=1e-2,
            report=None):
    """3D search: the same rules with the oracle's 3D window (references depth-major,
    indices volume positions) and per-slab norms."""
    v64 = np.asarray(v, dtype=np.float64)
    q, H, W = v64.shape
    Z = q - d + 1
    N = np.stack([O.patch_norms(v64[z:z + d], P) for z in range(Z)])
    rl = O.ref_list(H, W, P, s)
    n2 = len(rl)
    sel = np.arange(Z * n2) if refs is None else np.asarray(refs)
    gpu_idx = np.asarray(gpu_idx)
    gpu_dist = np.asarray(gpu_dist)
    rep = report or ParityReport()

    def norm_of(m):
        zc, rem = divmod(int(m), H * W)
        return N[zc, rem // W, rem % W]

    for row, i in enumerate(sel):
        z, i2 = divmod(int(i), n2)
        ry, rx = int(rl[i2, 0]), int(rl[i2, 1])
        dd, jj = O.window3d_distances(v64, P, d, Wn, c, z, ry, rx)
        _check_row(rep, i, dd, jj, K, gpu_idx[row], gpu_dist[row], N[z, ry, rx], norm_of, tol,
                   floor)
    return rep


def check_exact(gpu_idx, gpu_dist, oidx, odist):
    """Bit-exact comparison for integer-valued inputs where float32 arithmetic is exact."""
    assert np.array_equal(np.asarray(gpu_idx), oidx)
    assert np.array_equal(np.asarray(gpu_dist).astype(np.float64), odist)


# NCC tolerance on e = 2 - 2 NCC (absolute): float32 accumulation of n = P*P*C products
# errs by at most n*u*||X_i||*||X_j|| (Cauchy-Schwarz), the reciprocal norms by a few u
# each, so |de| <= 2 (n + 8) u ~ 3.1e-5 at n = 256; the float16 split adds its ~2^-22
# residual.  The bfloat16 split computes the NCC of the patches rounded to 16 significant
# bits exactly (all four products, norms of the rounded values): rounding moves each
# unit-normalised patch by at most 2^-15, so e = ||u_i - u_j||^2 <= 4 moves by at most
# 2 * 2 * 2 * 2^-15 ~ 1.2e-4, and 2e-4 covers that plus the float32 part.
NCC_TOL = {"fp32": 4e-5, "fp16x3": 4e-5, "bf16x4": 2e-4}


def check_ncc(x, P, s, Wn, K, gpu_idx, gpu_dist, refs=None, tol=4e-5, report=None):
    """NCC rows (e = 2 - 2 NCC) against the oracle: |e_gpu - e*| <= tol per returned pair,
    and the set rule with tau = tol around the oracle's K-th value."""
    x64 = np.asarray(x, dtype=np.float64)
    if x64.ndim == 2:
        x64 = x64[None]
    C, H, W = x64.shape
    rl = O.ref_list(H, W, P, s)
    sel = np.arange(len(rl)) if refs is None else np.asarray(refs)
    gpu_idx = np.asarray(gpu_idx)
    gpu_dist = np.asarray(gpu_dist)
    rep = report or ParityReport()
    for row, i in enumerate(sel):
        ry, rx = int(rl[i, 0]), int(rl[i, 1])
        ncc, j = O.window_ncc(x64, P, Wn, ry, rx)
        e = 2.0 - 2.0 * ncc
        oidx, odist = O.select_k(e, j, K)
        lookup = dict(zip(j.tolist(), e.tolist()))
        gi, gd = gpu_idx[row], gpu_dist[row]
        rep.n_refs += 1
        kk = min(K, e.size)
        if np.any(gi[kk:] != -1) or np.any(np.isfinite(gd[kk:])):
            rep.tolerant_mismatch += 1
            rep.messages.append(f"ref {i}: bad padding")
            continue
        members = gi[:kk].tolist()
        if len(set(members)) != kk or any(m not in lookup for m in members):
            rep.tolerant_mismatch += 1
            rep.messages.append(f"ref {i}: non-candidate or duplicate indices")
            continue
        estar = np.array([lookup[m] for m in members])
        err = np.abs(gd[:kk].astype(np.float64) - estar)
        rep.rel.append(err)
        if np.any(err > tol):
            rep.tolerant_mismatch += 1
            rep.messages.append(f"ref {i}: error {err.max():.3e}")
        keys = list(zip(gd[:kk].tolist(), members))
        if keys != sorted(keys):
            rep.order_violations += 1
        t = odist[kk - 1]
        if set(members) != set(oidx[:kk].tolist()):
            rep.strict_mismatch += 1
            must = {int(a) for a, b in zip(j, e) if b < t - tol}
            if np.any(estar > t + tol) or not must.issubset(set(members)):
                rep.tolerant_mismatch += 1
                rep.messages.append(f"ref {i}: set rule violated")
    return rep


# ---------------------------------------------------------------------------------------
# Whole-image parity from a cached oracle table.  The oracle's sorted head of every
# reference (its K + EXTRA smallest (d*, j) under the (d, j) key, the candidate count, the
# reference norm and the norms of the head's candidates) holds everything the distance
# and set rules look at: the set rule's forced members (d* < t - tau) are oracle top-K
# entries, and a GPU member outside the head has d* >= the head's last distance, so it
# breaks the rule unless the head's last distance is itself within t + tau (then that
# reference is checked against its full window instead).
EXTRA = 16


def _head_rows(args):
    x64, P, Wn, K, pos = args
    out = []
    for ry, rx in pos:
        d, j = O.window_distances(x64, P, Wn, int(ry), int(rx))
        hj, hd = O.select_k(d, j, K + EXTRA)
        out.append((d.size, hj, hd))
    return out


class OracleHead:
    """Oracle heads of a set of references of one image (computed once, reused by every
    form compared against it)."""

    def __init__(self, x, P, s, Wn, K, refs=None):
        x64 = np.asarray(x, dtype=np.float64)
        if x64.ndim == 2:
            x64 = x64[None]
        self.x64, self.P, self.s, self.Wn, self.K = x64, P, s, Wn, K
        C, H, W = x64.shape
        self.N = O.patch_norms(x64, P)
        self.rl = O.ref_list(H, W, P, s)
        self.refs = np.arange(len(self.rl)) if refs is None else np.asarray(refs)
        pos = self.rl[self.refs]
        parts = [_head_rows((x64, P, Wn, K, pos))]
        rows = [r for p in parts for r in p]
        self.ncand = np.array([r[0] for r in rows])
        self.hj = np.stack([r[1] for r in rows])
        self.hd = np.stack([r[2] for r in rows])
        self.ni = self.N[pos[:, 0], pos[:, 1]]
        jj = np.maximum(self.hj, 0)
        self.hn = np.where(self.hj >= 0, self.N[jj // W, jj % W], 0.0)

    def check(self, gpu_idx, gpu_dist, tol=1e-4, floor=1e-2, report=None):
        """Rows of the GPU result for self.refs (gpu_idx[self.refs] etc. already taken)."""
        K = self.K
        rep = report or ParityReport()
        W = self.x64.shape[2]
        for row, i in enumerate(self.refs):
            gi, gd = np.asarray(gpu_idx[row]), np.asarray(gpu_dist[row])
            kk = min(K, int(self.ncand[row]))
            hj, hd, hn = self.hj[row], self.hd[row], self.hn[row]
            t = hd[kk - 1]
            tau = tol * max(t, floor * (self.ni[row] + hn[kk - 1]))
            head_ok = kk < K or not (hd[-1] <= t + tau)  # the head covers every d* <= t + tau
            members = gi[:kk].tolist()
            pos = {int(j): q for q, j in enumerate(hj.tolist()) if j >= 0}
            if not head_ok or any(m not in pos for m in members):
                # outside the head (or a head too short for the band): full window
                ry, rx = self.rl[i]
                d, j = O.window_distances(self.x64, self.P, self.Wn, int(ry), int(rx))
                N = self.N
                _check_row(rep, i, d, j, K, gi, gd, self.ni[row],
                           lambda m: N[m // W, m % W], tol, floor)
                continue
            rep.n_refs += 1
            if np.any(gi[kk:] != -1) or np.any(np.isfinite(gd[kk:])):
                rep.tolerant_mismatch += 1
                rep.messages.append(f"ref {i}: bad padding")
                continue
            if len(set(members)) != kk:
                rep.tolerant_mismatch += 1
                rep.messages.append(f"ref {i}: duplicate indices {members}")
                continue
            q = np.array([pos[m] for m in members])
            dstar = hd[q]
            rel = np.abs(gd[:kk].astype(np.float64) - dstar) / np.maximum(dstar, floor * (self.ni[row] + hn[q]))
            rep.rel.append(rel)
            if np.any(rel > tol):
                rep.tolerant_mismatch += 1
                rep.messages.append(f"ref {i}: rel error {rel.max():.3e}")
            keys = list(zip(gd[:kk].tolist(), members))
            if keys != sorted(keys):
                rep.order_violations += 1
            if set(members) != set(hj[:kk].tolist()):
                rep.strict_mismatch += 1
                must = {int(a) for a, b in zip(hj[:kk], hd[:kk]) if b < t - tau}
                if np.any(dstar > t + tau) or not must.issubset(set(members)):
                    rep.tolerant_mismatch += 1
                    rep.messages.append(f"ref {i}: set rule violated")
        return rep
