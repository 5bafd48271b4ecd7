"""FP64 CPU oracle for block matching (BM) -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this
module. The product path (the HIP library and its Python binding) never calls it and
shares no code with it.

What it computes is the plain definition of block matching, written out slowly:

* Euclidean BM (Sec. III-A, Eq. ``equ:bm`` with the metric of Eq. ``equ:bmMetric_app``):
  for every reference patch X_i, the distance to a candidate X_j is the per-pair
  subtraction sum_{c,l,m} (X_j - X_i)^2, evaluated in float64; the K candidates with the
  smallest distance form the set S_i, |S_i| <= K.
* Multi-channel patches are joint sqrt(n) x sqrt(n) x p blocks and the distance sums over
  channels (Sec. IV, the channel sum S(.) of Eq. ``equ:self-convMM``).
* The candidates of X_i are the patches inside its search window Omega_i (footnote to
  Eq. ``eq:unifySelfConv``).

Readings taken where the paper is silent (each one is listed in the design notes):

* the window of side Wn holds the candidate top-left offsets (dy, dx) in [-a, b]^2 with
  a = floor(Wn / 2) and b = Wn - 1 - a: [-r, r]^2, r = (Wn - 1) / 2, for odd Wn, and
  [-Wn/2, Wn/2 - 1]^2 for even Wn (the paper's 30 x 30), so N_s = Wn^2 candidates away
  from borders;
* at image borders the window is intersected with the valid positions, never shifted;
* references sit on the grid {0, s, 2s, ...} in each axis (the last row/column is not
  forced in); candidates use stride 1 (all overlapping patches);
* a reference is its own candidate (distance 0; Sec. IV footnote on the group order);
* ties are broken by the candidate's linear index j = qy * W + qx, i.e. the result is
  the first K entries of the candidates sorted by the key (d, j);
* fewer than K candidates: the row is padded with index -1 and distance +inf.

* Normalized-cross-correlation BM (Sec. III-A, Eq. ``equ:cor``; Lemma 1; Theorem 1 item 3):
  the K candidates with the largest vec(X_j)^T vec(X_i) / (||X_j||_F ||X_i||_F).  The
  oracle reports them through the equivalent distance e = 2 - 2 NCC (the squared distance
  between the unit-normalised patches), so the same ascending (e, j) order and padding
  apply.  Reading: when either patch has zero norm its NCC is taken as 0 (e = 2).
* Non-local means (Sec. III-A, Eq. ``equ:nlm``; Prop. 1): for every reference X_i, the
  weights s_i(j) = exp(-||X_j - X_i||^2 / b^2) / Theta_i over the candidates of its search
  window, Theta_i their unnormalised sum, and the recovered patch sum_j s_i(j) X_j.  The
  oracle returns Theta_i and the recovered patch (C x P x P) per reference.
* 3D block matching (Sec. IV, 3D Self-Convolution; the multi-channel runtime setup of
  Sec. V): the volume has q channels (frames, modalities); a patch is a d x P x P block
  (d <= q consecutive channels) and the search window is Wn x Wn x c, so candidates also
  come from other channel positions.  Readings: reference depths are every position
  z = 0..q-d, spatial references on the stride-s grid as in 2D; the depth window holds the
  c positions z - floor((c-1)/2) .. z - floor((c-1)/2) + c - 1 (c = 9: z-4..z+4; c = 2: z,
  z+1), intersected with 0..q-d, never shifted; the candidate index is
  j = (z' H + qy) W + qx and references are numbered depth-major, z * n_ref2d + (grid index);
  ties and padding as in 2D.  c = 1 with d = q is plain multi-channel BM.
* Group gather and aggregation (Sec. IV, image reconstruction): the group of reference i is
  Y_i = [X_{S_i(1)}, ..., X_{S_i(K)}] (padding entries give zero patches); aggregation
  deposits every group patch back at its location S_i(k), summing over overlaps, and
  divides each pixel by the number of deposited patches covering it (0 where none does).

Parity status: every function below is pinned by the CPU test suite against hand-checked
values, closed forms, library routines or brute force (see tests/test_oracle_pins.py).
"""
from __future__ import annotations

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

PAD_INDEX = -1


# --------------------------------------------------------------------------------------
# Geometry (readings: reference grid, clipped window)
# --------------------------------------------------------------------------------------
def valid_extent(H: int, W: int, P: int):
    """Number of valid patch positions per axis: sqrt(M) = sqrt(N) - sqrt(n) + 1 (Eq. eq:selfConv)."""
    return H - P + 1, W - P + 1


def ref_positions(H: int, W: int, P: int, s: int):
    """Reference top-left rows and columns on the stride-s grid {0, s, 2s, ...}."""
    Hv, Wv = valid_extent(H, W, P)
    return np.arange(0, Hv, s), np.arange(0, Wv, s)


def ref_list(H: int, W: int, P: int, s: int):
    """All references in row-major grid order as an (n_ref, 2) array of (ry, rx)."""
    ys, xs = ref_positions(H, W, P, s)
    yy, xx = np.meshgrid(ys, xs, indexing="ij")
    return np.stack([yy.ravel(), xx.ravel()], axis=1)


def window_offsets(Wn: int):
    """Smallest and largest candidate offset per axis of a window of side Wn: -floor(Wn/2)
    and Wn - 1 - floor(Wn/2) (equal magnitudes for odd Wn; one fewer after than before the
    reference for even Wn)."""
    a = Wn // 2
    return -a, Wn - 1 - a


def window_box(ry: int, rx: int, Hv: int, Wv: int, Wn: int):
    """Inclusive candidate box of reference (ry, rx): the Wn x Wn offsets clipped to the image."""
    lo, hi = window_offsets(Wn)
    return max(0, ry + lo), min(Hv - 1, ry + hi), max(0, rx + lo), min(Wv - 1, rx + hi)


def candidate_count(H: int, W: int, P: int, s: int, Wn: int) -> int:
    """Total number of (reference, candidate) pairs, by enumeration of every reference."""
    Hv, Wv = valid_extent(H, W, P)
    total = 0
    for ry, rx in ref_list(H, W, P, s):
        y0, y1, x0, x1 = window_box(int(ry), int(rx), Hv, Wv, Wn)
        total += (y1 - y0 + 1) * (x1 - x0 + 1)
    return total


# --------------------------------------------------------------------------------------
# Patch norms (h_X (.) h_X, Sec. III-B; used by Lemma 2)
# --------------------------------------------------------------------------------------
def patch_norms(x: np.ndarray, P: int) -> np.ndarray:
    """Squared Frobenius norm of every valid patch, summed over channels, float64.

    N[y, x] = sum_c sum_{l<P} sum_{m<P} X_c[y+l, x+m]^2 -- the entries of h_X (.) h_X.
    """
    x = np.asarray(x, dtype=np.float64)
    C, H, W = x.shape
    Hv, Wv = valid_extent(H, W, P)
    sq = x * x
    out = np.zeros((Hv, Wv), dtype=np.float64)
    for c in range(C):
        for l in range(P):
            for m in range(P):
                out += sq[c, l:l + Hv, m:m + Wv]
    return out


# --------------------------------------------------------------------------------------
# Distances by per-pair subtraction (Eq. equ:bmMetric_app)
# --------------------------------------------------------------------------------------
def pair_distance(x: np.ndarray, P: int, ry: int, rx: int, qy: int, qx: int) -> float:
    """||X_j - X_i||_F^2 for reference (ry, rx) and candidate (qy, qx), float64."""
    x = np.asarray(x, dtype=np.float64)
    diff = x[:, qy:qy + P, qx:qx + P] - x[:, ry:ry + P, rx:rx + P]
    return float(np.sum(diff * diff))


def window_distances(x64: np.ndarray, P: int, Wn: int, ry: int, rx: int):
    """All in-window distances of one reference.

    Returns (d, j): float64 distances and int64 candidate indices j = qy*W + qx, both
    flattened in row-major window order.
    """
    C, H, W = x64.shape
    Hv, Wv = valid_extent(H, W, P)
    y0, y1, x0, x1 = window_box(ry, rx, Hv, Wv, Wn)
    region = x64[:, y0:y1 + P, x0:x1 + P]
    cands = sliding_window_view(region, (P, P), axis=(1, 2))  # C, ny, nx, P, P
    ref = x64[:, ry:ry + P, rx:rx + P]
    diff = cands - ref[:, None, None, :, :]
    d = np.sum(diff * diff, axis=(0, 3, 4))  # ny, nx
    qy = np.arange(y0, y1 + 1)[:, None]
    qx = np.arange(x0, x1 + 1)[None, :]
    j = qy * W + qx
    return d.ravel(), np.broadcast_to(j, d.shape).ravel().astype(np.int64)


def select_k(d: np.ndarray, j: np.ndarray, K: int):
    """The K smallest candidates under the key (d, j), padded with (-1, +inf)."""
    order = np.lexsort((j, d))[:K]
    idx = np.full(K, PAD_INDEX, dtype=np.int64)
    dist = np.full(K, np.inf, dtype=np.float64)
    idx[:order.size] = j[order]
    dist[:order.size] = d[order]
    return idx, dist


def bm(x: np.ndarray, P: int, s: int, Wn: int, K: int, refs=None):
    """Euclidean block matching (Eq. equ:bm), float64 brute force.

    ``x`` is C x H x W (any real dtype; promoted exactly to float64). ``refs`` optionally
    selects reference numbers (row-major grid order); by default every reference is done.
    Returns (idx [n, K] int64, dist [n, K] float64), rows sorted ascending by (d, j).
    """
    x64 = np.asarray(x, dtype=np.float64)
    if x64.ndim == 2:
        x64 = x64[None]
    C, H, W = x64.shape
    rl = ref_list(H, W, P, s)
    sel = np.arange(len(rl)) if refs is None else np.asarray(refs, dtype=np.int64)
    idx = np.empty((len(sel), K), dtype=np.int64)
    dist = np.empty((len(sel), K), dtype=np.float64)
    for n, i in enumerate(sel):
        ry, rx = int(rl[i, 0]), int(rl[i, 1])
        d, j = window_distances(x64, P, Wn, ry, rx)
        idx[n], dist[n] = select_k(d, j, K)
    return idx, dist


# --------------------------------------------------------------------------------------
# Normalized cross-correlation (Eq. equ:cor, Lemma 1)
# --------------------------------------------------------------------------------------
def window_ncc(x64: np.ndarray, P: int, Wn: int, ry: int, rx: int):
    """NCC of one reference with every in-window candidate.

    Returns (ncc, j) in row-major window order: the inner product of the vectorised patches
    divided by the product of their Frobenius norms, float64; 0 when a norm is 0.
    """
    C, H, W = x64.shape
    Hv, Wv = valid_extent(H, W, P)
    y0, y1, x0, x1 = window_box(ry, rx, Hv, Wv, Wn)
    cands = sliding_window_view(x64[:, y0:y1 + P, x0:x1 + P], (P, P), axis=(1, 2))
    ref = x64[:, ry:ry + P, rx:rx + P]
    dot = np.sum(cands * ref[:, None, None, :, :], axis=(0, 3, 4))
    nq = np.sqrt(np.sum(cands * cands, axis=(0, 3, 4)))
    npp = np.sqrt(np.sum(ref * ref))
    den = nq * npp
    ncc = np.where(den > 0, dot / np.where(den > 0, den, 1.0), 0.0)
    j = (np.arange(y0, y1 + 1)[:, None] * W + np.arange(x0, x1 + 1)[None, :])
    return ncc.ravel(), np.broadcast_to(j, ncc.shape).ravel().astype(np.int64)


def bm_ncc(x: np.ndarray, P: int, s: int, Wn: int, K: int, refs=None):
    """NCC block matching (Eq. equ:cor), float64 brute force.

    Same arguments and layout as ``bm``; the returned distances are e = 2 - 2 NCC, rows
    sorted ascending by (e, j), i.e. descending NCC with ties by the smaller index.
    """
    x64 = np.asarray(x, dtype=np.float64)
    if x64.ndim == 2:
        x64 = x64[None]
    C, H, W = x64.shape
    rl = ref_list(H, W, P, s)
    sel = np.arange(len(rl)) if refs is None else np.asarray(refs, dtype=np.int64)
    idx = np.empty((len(sel), K), dtype=np.int64)
    dist = np.empty((len(sel), K), dtype=np.float64)
    for n, i in enumerate(sel):
        ry, rx = int(rl[i, 0]), int(rl[i, 1])
        ncc, j = window_ncc(x64, P, Wn, ry, rx)
        idx[n], dist[n] = select_k(2.0 - 2.0 * ncc, j, K)
    return idx, dist


# --------------------------------------------------------------------------------------
# Non-local means (Eq. equ:nlm, Prop. 1)
# --------------------------------------------------------------------------------------
def nlm(x: np.ndarray, P: int, s: int, Wn: int, b: float, refs=None):
    """NLM weights over each reference's window, float64.

    Returns (theta [n], patch [n, C, P, P]): Theta_i = sum_j exp(-d_ij / b^2) and the
    weighted average sum_j s_i(j) X_j with s_i(j) = exp(-d_ij / b^2) / Theta_i, the d_ij
    being the per-pair subtraction distances of ``window_distances``.
    """
    x64 = np.asarray(x, dtype=np.float64)
    if x64.ndim == 2:
        x64 = x64[None]
    C, H, W = x64.shape
    Hv, Wv = valid_extent(H, W, P)
    rl = ref_list(H, W, P, s)
    sel = np.arange(len(rl)) if refs is None else np.asarray(refs, dtype=np.int64)
    theta = np.empty(len(sel), dtype=np.float64)
    patch = np.empty((len(sel), C, P, P), dtype=np.float64)
    for n, i in enumerate(sel):
        ry, rx = int(rl[i, 0]), int(rl[i, 1])
        d, _ = window_distances(x64, P, Wn, ry, rx)
        w = np.exp(-d / (b * b))
        y0, y1, x0, x1 = window_box(ry, rx, Hv, Wv, Wn)
        cands = sliding_window_view(x64[:, y0:y1 + P, x0:x1 + P], (P, P), axis=(1, 2))
        cands = cands.transpose(1, 2, 0, 3, 4).reshape(-1, C, P, P)  # row-major window order
        theta[n] = w.sum()
        patch[n] = np.tensordot(w, cands, axes=(0, 0)) / theta[n]
    return theta, patch


# --------------------------------------------------------------------------------------
# Group gather and aggregation (Sec. IV, image reconstruction)
# --------------------------------------------------------------------------------------
def gather_groups(x: np.ndarray, idx: np.ndarray, P: int) -> np.ndarray:
    """Y_i for every row of ``idx`` [n, K]: groups [n, K, C, P, P], zero for index -1."""
    x64 = np.asarray(x, dtype=np.float64)
    C, H, W = x64.shape
    n, K = idx.shape
    out = np.zeros((n, K, C, P, P), dtype=np.float64)
    for i in range(n):
        for k in range(K):
            j = int(idx[i, k])
            if j < 0:
                continue
            qy, qx = j // W, j % W
            out[i, k] = x64[:, qy:qy + P, qx:qx + P]
    return out


def aggregate_groups(groups: np.ndarray, idx: np.ndarray, C: int, H: int, W: int):
    """Deposit every group patch at its location and normalise by the coverage count.

    Returns (image [C, H, W] float64, count [H, W] int64); pixels no patch covers are 0.
    """
    n, K = idx.shape
    P = groups.shape[-1]
    acc = np.zeros((C, H, W), dtype=np.float64)
    cnt = np.zeros((H, W), dtype=np.int64)
    for i in range(n):
        for k in range(K):
            j = int(idx[i, k])
            if j < 0:
                continue
            qy, qx = j // W, j % W
            acc[:, qy:qy + P, qx:qx + P] += groups[i, k]
            cnt[qy:qy + P, qx:qx + P] += 1
    out = np.where(cnt > 0, acc / np.maximum(cnt, 1), 0.0)
    return out, cnt


# --------------------------------------------------------------------------------------
# 3D block matching (Sec. IV, 3D Self-Convolution)
# --------------------------------------------------------------------------------------
def depth_window(z: int, Z: int, c: int):
    """Inclusive depth range of the candidates of a reference at depth z (Z = q - d + 1)."""
    lo = z - (c - 1) // 2
    return max(0, lo), min(Z - 1, lo + c - 1)


def window3d_distances(v64: np.ndarray, P: int, d: int, Wn: int, c: int, z: int, ry: int, rx: int):
    """All in-window distances of the reference (z, ry, rx): per-pair subtraction over the
    d x P x P blocks, float64.  Returns (dist, j), slab-major then row-major."""
    q, H, W = v64.shape
    Hv, Wv = valid_extent(H, W, P)
    z0, z1 = depth_window(z, q - d + 1, c)
    y0, y1, x0, x1 = window_box(ry, rx, Hv, Wv, Wn)
    ref = v64[z:z + d, ry:ry + P, rx:rx + P]
    qy = np.arange(y0, y1 + 1)[:, None]
    qx = np.arange(x0, x1 + 1)[None, :]
    ds, js = [], []
    for zc in range(z0, z1 + 1):
        cands = sliding_window_view(v64[zc:zc + d, y0:y1 + P, x0:x1 + P], (P, P), axis=(1, 2))
        diff = cands - ref[:, None, None, :, :]
        dd = np.sum(diff * diff, axis=(0, 3, 4))
        ds.append(dd.ravel())
        js.append(np.broadcast_to((zc * H + qy) * W + qx, dd.shape).ravel().astype(np.int64))
    return np.concatenate(ds), np.concatenate(js)


def bm3d(v: np.ndarray, P: int, d: int, s: int, Wn: int, c: int, K: int, refs=None):
    """3D Euclidean block matching over a q x H x W volume, float64 brute force.

    Returns (idx [n, K] int64, dist [n, K] float64) for the references numbered depth-major
    (all (q - d + 1) * n_ref2d of them, or the numbers in ``refs``)."""
    v64 = np.asarray(v, dtype=np.float64)
    q, H, W = v64.shape
    if not 1 <= d <= q:
        raise ValueError("patch depth must be in [1, q]")
    rl = ref_list(H, W, P, s)
    n2 = len(rl)
    n = (q - d + 1) * n2
    sel = np.arange(n) if refs is None else np.asarray(refs, dtype=np.int64)
    idx = np.empty((len(sel), K), dtype=np.int64)
    dist = np.empty((len(sel), K), dtype=np.float64)
    for m, i in enumerate(sel):
        z, i2 = divmod(int(i), n2)
        dd, jj = window3d_distances(v64, P, d, Wn, c, z, int(rl[i2, 0]), int(rl[i2, 1]))
        idx[m], dist[m] = select_k(dd, jj, K)
    return idx, dist


def bm_two_image(x: np.ndarray, y: np.ndarray, P: int, s: int, Wn: int, K: int):
    """BM of the reference patches of ``x`` against candidate patches of ``y`` (same shape).

    The windowed Self-Convolution X_{Omega_i} * X_i with the sub-image taken from a second
    image; used to check offset recovery on shifted copies.
    """
    x64 = np.asarray(x, dtype=np.float64)
    y64 = np.asarray(y, dtype=np.float64)
    C, H, W = x64.shape
    Hv, Wv = valid_extent(H, W, P)
    rl = ref_list(H, W, P, s)
    idx = np.empty((len(rl), K), dtype=np.int64)
    dist = np.empty((len(rl), K), dtype=np.float64)
    for n, (ry, rx) in enumerate(rl):
        ry, rx = int(ry), int(rx)
        y0, y1, x0, x1 = window_box(ry, rx, Hv, Wv, Wn)
        cands = sliding_window_view(y64[:, y0:y1 + P, x0:x1 + P], (P, P), axis=(1, 2))
        ref = x64[:, ry:ry + P, rx:rx + P]
        diff = cands - ref[:, None, None, :, :]
        d = np.sum(diff * diff, axis=(0, 3, 4))
        j = (np.arange(y0, y1 + 1)[:, None] * W + np.arange(x0, x1 + 1)[None, :])
        idx[n], dist[n] = select_k(d.ravel(), np.broadcast_to(j, d.shape).ravel(), K)
    return idx, dist
