"""FP64 CPU oracle for LeaFi-enhanced tree search.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the GPU library (no kernels, headers, helpers or constant tables) and reads
nothing the GPU library produced: every input comes from `workloads`.

Each function states the passage of the paper it follows (LeaFi, Wang,
Ileana and Palpanas, SIGMOD 2025).  Where the paper is silent the function
says which reading it takes; the readings are listed in the design notes.
Everything is plain NumPy in FP64 (plus the C brute force in bruteforce.c for
the distance scans), with no blocking or reordering beyond what the
definitions state.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_BF_SO = os.path.join(_HERE, "_bruteforce.so")
_bf = None


def build_bruteforce(force: bool = False) -> str:
    """Compile bruteforce.c (gcc -O2, OpenMP, no fast-math) into oracle/_bruteforce.so."""
    src = os.path.join(_HERE, "bruteforce.c")
    if force or not os.path.exists(_BF_SO) or os.path.getmtime(_BF_SO) < os.path.getmtime(src):
        import subprocess
        tmp = _BF_SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, _BF_SO)
    return _BF_SO


def _lib():
    global _bf
    if _bf is None:
        build_bruteforce()
        lib = ctypes.CDLL(_BF_SO)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I32 = ctypes.c_int32
        lib.or_znorm.argtypes = [P, I64, I32, P]
        lib.or_knn.argtypes = [P, I64, I32, P, I64, I32, P, P]
        lib.or_leaf_knn.argtypes = [P, P, P, I32, I32, P, I64, I32, P, P]
        lib.or_num_threads.restype = ctypes.c_int
        lib.or_set_num_threads.argtypes = [ctypes.c_int]
        _bf = lib
    return _bf


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_lib().or_num_threads())


def set_num_threads(n: int) -> None:
    """Host threads of the C brute force's parallel loops from now on."""
    _lib().or_set_num_threads(int(n))


# ---------------------------------------------------------------------------
# z-normalisation and distances (Section "Preliminaries")
# ---------------------------------------------------------------------------

def znorm(x: np.ndarray) -> np.ndarray:
    """Stored z-normalised series: fp32((x - mu) / sigma), mu and population sigma in FP64.

    Reading: population standard deviation; a series with sigma < 1e-8 is
    stored as all zeros; the index keeps the normalised values as fp32.
    """
    x = np.ascontiguousarray(x, dtype=np.float32)
    n, m = x.shape
    out = np.empty_like(x)
    _lib().or_znorm(_ptr(x), n, m, _ptr(out))
    return out


def znorm_py(x: np.ndarray) -> np.ndarray:
    """The same definition in NumPy (used to pin the C version on small inputs)."""
    x64 = np.asarray(x, dtype=np.float64)
    mu = x64.mean(axis=1, keepdims=True)
    sd = np.sqrt(((x64 - mu) ** 2).mean(axis=1, keepdims=True))
    z = np.where(sd < 1e-8, 0.0, (x64 - mu) / np.where(sd < 1e-8, 1.0, sd))
    return z.astype(np.float32)


def knn(data_s: np.ndarray, q_s: np.ndarray, k: int):
    """Exact k-NN by brute force: ids [nq, k] int64 and Euclidean d [nq, k] FP64, by (d, id)."""
    data_s = np.ascontiguousarray(data_s, dtype=np.float32)
    q_s = np.ascontiguousarray(q_s, dtype=np.float32)
    n, m = data_s.shape
    nq = q_s.shape[0]
    ids = np.empty((nq, k), dtype=np.int64)
    d = np.empty((nq, k), dtype=np.float64)
    _lib().or_knn(_ptr(data_s), n, m, _ptr(q_s), nq, k, _ptr(ids), _ptr(d))
    return ids, d


def knn_stream(chunks, q_s: np.ndarray, k: int):
    """Exact k-NN over a collection given in consecutive raw chunks (an iterable
    of (first row id, raw fp32 rows)): each chunk is z-normalised (znorm) and
    searched by brute force (knn), and the running k best are kept by (d, id).
    The same result as knn over the whole normalised collection; for
    collections too large to hold normalised on the host at once."""
    q_s = np.ascontiguousarray(q_s, dtype=np.float32)
    nq = q_s.shape[0]
    best_d = np.full((nq, k), np.inf)
    best_i = np.full((nq, k), -1, dtype=np.int64)
    for lo, raw in chunks:
        ids, d = knn(znorm(raw), q_s, min(k, len(raw)))
        cat_d = np.concatenate([best_d, d], axis=1)
        cat_i = np.concatenate([best_i, ids + lo], axis=1)
        # (d, id) order; empty slots (+inf, -1) sort last
        key_i = np.where(cat_i < 0, np.iinfo(np.int64).max, cat_i)
        o = np.lexsort((key_i, cat_d), axis=1)[:, :k]
        best_d = np.take_along_axis(cat_d, o, axis=1)
        best_i = np.take_along_axis(cat_i, o, axis=1)
    return best_i, best_d


def leaf_knn(data_s: np.ndarray, leaves: list, q_s: np.ndarray, k: int):
    """Per-leaf exact k-NN: d [nq, N, k] and ids [nq, N, k]; d[:, L, 0] is d^L(q, L)."""
    order = np.concatenate(leaves).astype(np.int64)
    off = np.zeros(len(leaves) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(l) for l in leaves])
    packed = np.ascontiguousarray(data_s[order], dtype=np.float32)
    q_s = np.ascontiguousarray(q_s, dtype=np.float32)
    nq, m = q_s.shape
    N = len(leaves)
    ids = np.empty((nq, N, k), dtype=np.int64)
    d = np.empty((nq, N, k), dtype=np.float64)
    _lib().or_leaf_knn(_ptr(packed), _ptr(order), _ptr(off), N, m, _ptr(q_s), nq, k, _ptr(ids), _ptr(d))
    return d, ids


# ---------------------------------------------------------------------------
# Tree index with EAPCA-style node summaries (Section "Preliminaries",
# tree-based indexes; DSTree backbone)
# ---------------------------------------------------------------------------

def segments(m: int, S: int):
    """Equal segments: segment s covers [floor(s*m/S), floor((s+1)*m/S))."""
    b = [(s * m) // S for s in range(S + 1)]
    return [(b[s], b[s + 1]) for s in range(S)]


def segment_stats(xs: np.ndarray, S: int):
    """Per-series, per-segment mean and population std of the stored fp32 values.

    Computed in FP64 and kept as fp32 (the form the summaries are stored in).
    Returns (mu [n, S] fp32, sd [n, S] fp32).
    """
    n, m = xs.shape
    mu = np.empty((n, S), dtype=np.float32)
    sd = np.empty((n, S), dtype=np.float32)
    for s, (a, b) in enumerate(segments(m, S)):
        seg = xs[:, a:b].astype(np.float64)
        mseg = seg.mean(axis=1)
        mu[:, s] = mseg
        sd[:, s] = np.sqrt(((seg - mseg[:, None]) ** 2).mean(axis=1))
    return mu, sd


@dataclass
class Node:
    members: np.ndarray               # ids, ascending
    left: "Node | None" = None
    right: "Node | None" = None
    leaf_id: int = -1
    split: tuple = ()                 # (segment, stat, rule, value or count)


@dataclass
class Tree:
    root: Node
    leaves: list = field(default_factory=list)   # list of id arrays (ascending), DFS order
    S: int = 16
    m: int = 0


def build_tree(mu: np.ndarray, sd: np.ndarray, m: int, capacity: int, rule: str = "median") -> Tree:
    """Binary tree over the summaries, split until every leaf holds <= capacity series.

    Reading of the DSTree backbone (the paper gives no internals): a node over
    capacity splits on the (segment, statistic) pair with the largest
    seg_len * (max - min)^2 among its members (ties: lowest 2*segment + stat,
    stat 0 = mean, 1 = std).  `median` sends the first ceil(n/2) members in
    (value, id) order left; `midpoint` sends members with value <= (min+max)/2
    left, falling back to the median when one side would be empty.  Leaves are
    numbered in depth-first order, left child first.
    """
    n, S = mu.shape
    seglen = np.array([b - a for a, b in segments(m, S)], dtype=np.float64)
    stats = (mu.astype(np.float64), sd.astype(np.float64))
    root = Node(members=np.arange(n, dtype=np.int64))
    tree = Tree(root=root, S=S, m=m)
    # depth-first recursion, left child first, so leaf numbering is depth-first
    def visit(node: Node):
        ids = node.members
        if len(ids) <= capacity:
            node.leaf_id = len(tree.leaves)
            tree.leaves.append(ids)
            return
        best, best_key = -1.0, None
        for s in range(S):
            for st in range(2):
                v = stats[st][ids, s]
                score = seglen[s] * (v.max() - v.min()) ** 2
                if score > best:
                    best, best_key = score, (s, st)
        s, st = best_key
        v = stats[st][ids, s]
        left_mask = None
        if rule == "midpoint":
            mid = v.min() + (v.max() - v.min()) / 2.0
            left_mask = v <= mid
            if left_mask.all() or not left_mask.any():
                left_mask = None
        if left_mask is None:
            o = np.lexsort((ids, v))             # by value, then id
            nl = (len(ids) + 1) // 2
            left_mask = np.zeros(len(ids), dtype=bool)
            left_mask[o[:nl]] = True
            node.split = (s, st, "median", nl)
        else:
            node.split = (s, st, "midpoint", mid)
        node.left = Node(members=ids[left_mask])
        node.right = Node(members=ids[~left_mask])
        visit(node.left)
        visit(node.right)

    import sys
    old = sys.getrecursionlimit()
    sys.setrecursionlimit(max(old, 100000))
    try:
        visit(root)
    finally:
        sys.setrecursionlimit(old)
    return tree


def node_box(mu: np.ndarray, sd: np.ndarray, members: np.ndarray) -> np.ndarray:
    """Node summary: per segment [mu_lo, mu_hi, sd_lo, sd_hi] over the members, fp32.

    Bounds are widened outward by one fp32 ulp so that they contain the exact
    (unrounded) statistics of every member, which keeps the lower bound valid.
    """
    m_ = mu[members]
    s_ = sd[members]
    box = np.empty((mu.shape[1], 4), dtype=np.float32)
    box[:, 0] = np.nextafter(m_.min(axis=0), np.float32(-np.inf))
    box[:, 1] = np.nextafter(m_.max(axis=0), np.float32(np.inf))
    box[:, 2] = np.nextafter(s_.min(axis=0), np.float32(-np.inf))
    box[:, 3] = np.nextafter(s_.max(axis=0), np.float32(np.inf))
    return box


def leaf_boxes(mu, sd, tree: Tree) -> np.ndarray:
    return np.stack([node_box(mu, sd, ids) for ids in tree.leaves])


def query_stats(q_s: np.ndarray, S: int):
    """Per-segment mean and population std of stored queries, FP64 [nq, S] each."""
    nq, m = q_s.shape
    mu = np.empty((nq, S))
    sd = np.empty((nq, S))
    for s, (a, b) in enumerate(segments(m, S)):
        seg = q_s[:, a:b].astype(np.float64)
        mseg = seg.mean(axis=1)
        mu[:, s] = mseg
        sd[:, s] = np.sqrt(((seg - mseg[:, None]) ** 2).mean(axis=1))
    return mu, sd


def lower_bound(qmu: np.ndarray, qsd: np.ndarray, boxes: np.ndarray, m: int) -> np.ndarray:
    """Summary lower bound d^lb(q, N) for every query and node, FP64 [nq, N].

    For segment s of length l_s, the part of the squared distance inside the
    segment is at least l_s * ((mu_q - mu_x)^2 + (sd_q - sd_x)^2) (the cross
    term of the mean/deviation split vanishes and the deviation part obeys the
    reverse triangle inequality).  Replacing mu_x and sd_x by the node's range
    gives a bound for every member: the squared gap between the query value and
    the interval [lo, hi], summed with the segment weights.
    """
    S = boxes.shape[1]
    seglen = np.array([b - a for a, b in segments(m, S)], dtype=np.float64)
    b = boxes.astype(np.float64)
    gm = np.maximum(np.maximum(b[None, :, :, 0] - qmu[:, None, :], qmu[:, None, :] - b[None, :, :, 1]), 0.0)
    gs = np.maximum(np.maximum(b[None, :, :, 2] - qsd[:, None, :], qsd[:, None, :] - b[None, :, :, 3]), 0.0)
    return np.sqrt(((gm ** 2 + gs ** 2) * seglen[None, None, :]).sum(axis=2))


def visit_order(lb: np.ndarray) -> np.ndarray:
    """Leaves in the order the search visits them: ascending (d^lb, leaf id)."""
    nq, N = lb.shape
    ids = np.broadcast_to(np.arange(N), (nq, N))
    return np.lexsort((ids, lb), axis=1).astype(np.int32)


# ---------------------------------------------------------------------------
# iSAX backbone (Section "Preliminaries": SAX quantises each PAA value with
# discrete symbols, and iSAX compares words of different cardinalities, which
# makes them indexable in a prefix tree; Section "Evaluation Setup": MESSI,
# the in-memory iSAX index, is the paper's second backbone)
# ---------------------------------------------------------------------------

ISAX_MAX_BITS = 8  # symbols of up to 8 bits (cardinality 256) per segment


def isax_breakpoints(bits: int = ISAX_MAX_BITS) -> np.ndarray:
    """SAX breakpoints of cardinality 2^bits: the N(0, 1) quantiles
    Phi^-1(j / 2^bits), j = 1 .. 2^bits - 1, in FP64, kept as fp32 (reading:
    the PAA values they are compared with are stored as fp32).  Breakpoints of
    a smaller cardinality are a subset: those with j a multiple of
    2^(bits - b)."""
    from scipy.special import ndtri
    j = np.arange(1, 2 ** bits, dtype=np.float64)
    return ndtri(j / 2.0 ** bits).astype(np.float32)


def sax_symbols(mu: np.ndarray, bits: int = ISAX_MAX_BITS) -> np.ndarray:
    """SAX symbol of each PAA value (the segment means, fp32) at cardinality
    2^bits: the number of breakpoints <= the value (a value equal to a
    breakpoint takes the upper interval).  Symbols at b < bits bits are these
    shifted right by bits - b.  Returns int32, same shape as mu."""
    bp = isax_breakpoints(bits)
    return np.searchsorted(bp, np.asarray(mu, dtype=np.float32), side="right").astype(np.int32)


def build_isax_tree(mu: np.ndarray, m: int, capacity: int, max_bits: int = ISAX_MAX_BITS) -> Tree:
    """iSAX tree over the segment means (PAA), split until every leaf holds <=
    capacity series (or its members cannot be told apart at max_bits bits).

    Reading of the MESSI backbone (the paper names it, the iSAX papers define
    it): the root's children are the words of one bit per segment (each PAA
    value above or below 0), taken in ascending order of the word read with
    segment 0 as its highest bit.  A node over capacity takes one more bit of
    one segment: the segment (below max_bits) whose next bit divides the
    members most evenly, smallest |n0 - n1|, ties by the lowest segment.  If
    both halves are non-empty they become its children (the 0 half first);
    otherwise the node keeps all members with the refined symbol and tries
    again.  Leaves are numbered depth-first; members stay ascending by id.
    Each leaf records its bits and its symbol (at those bits) per segment in
    tree.isax[leaf] = (bits [S], symbol [S])."""
    n, S = mu.shape
    sym8 = sax_symbols(mu, max_bits).astype(np.int64)
    tree = Tree(root=Node(members=np.arange(n, dtype=np.int64)), S=S, m=m)
    tree.isax = []
    first = sym8 >> (max_bits - 1)
    words = np.zeros(n, dtype=np.int64)
    for s in range(S):
        words = (words << 1) | first[:, s]
    order = np.lexsort((np.arange(n), words))        # by word, then id
    uw, starts = np.unique(words[order], return_index=True)
    bounds = list(starts) + [n]

    def visit(ids, bits, sym):
        while len(ids) > capacity:
            elig = [s for s in range(S) if bits[s] < max_bits]
            if not elig:
                break                                  # identical at max_bits in every segment
            best, best_s, best_nb = None, -1, None
            for s in elig:
                nb = (sym8[ids, s] >> (max_bits - 1 - bits[s])) & 1
                n1 = int(nb.sum())
                d = abs(len(ids) - 2 * n1)
                if best is None or d < best:
                    best, best_s, best_nb = d, s, nb
            s = best_s
            bits = bits.copy()
            bits[s] += 1
            zero, one = ids[best_nb == 0], ids[best_nb == 1]
            if len(zero) and len(one):
                sz, so = sym.copy(), sym.copy()
                sz[s] = 2 * sym[s]
                so[s] = 2 * sym[s] + 1
                visit(zero, bits, sz)
                visit(one, bits, so)
                return
            sym = sym.copy()
            sym[s] = 2 * sym[s] + (0 if len(zero) else 1)
        tree.isax.append((bits.copy(), sym.copy()))
        tree.leaves.append(ids)

    for a, b in zip(bounds[:-1], bounds[1:]):
        ids = np.sort(order[a:b])
        visit(ids, np.ones(S, dtype=np.int64), first[ids[0]].copy())
    return tree


def isax_boxes(tree: Tree, max_bits: int = ISAX_MAX_BITS) -> np.ndarray:
    """Leaf summaries of an iSAX tree in the box form the lower bound takes:
    per segment the SAX interval of the leaf's symbol, [beta_c, beta_(c+1)]
    at its cardinality (-inf / +inf at the ends), widened outward by one fp32
    ulp (so it holds the exact segment mean of every member, not only the
    stored fp32 one), and the deviation unconstrained, [0, +inf].  With it the
    bound is MINDIST(PAA(q), iSAX word): the segment-weighted squared gaps
    between the query's segment means and the intervals."""
    bp = isax_breakpoints(max_bits)
    S = tree.S
    out = np.empty((len(tree.leaves), S, 4), dtype=np.float32)
    for L, (bits, sym) in enumerate(tree.isax):
        for s in range(S):
            step = 1 << (max_bits - int(bits[s]))
            c = int(sym[s])
            lo = bp[c * step - 1] if c > 0 else np.float32(-np.inf)
            hi = bp[(c + 1) * step - 1] if c + 1 < (1 << int(bits[s])) else np.float32(np.inf)
            out[L, s, 0] = np.nextafter(np.float32(lo), np.float32(-np.inf))
            out[L, s, 1] = np.nextafter(np.float32(hi), np.float32(np.inf))
            out[L, s, 2] = 0.0
            out[L, s, 3] = np.inf
    return out


# ---------------------------------------------------------------------------
# Learned filter: one-hidden-layer MLP (Section "Evaluation Setup", LeaFi
# instantiation: hidden width equal to the series length, ReLU)
# ---------------------------------------------------------------------------

def unpack_mlp(w: np.ndarray, m: int, h: int):
    """Split a packed filter [W1 (m*h, input-major) | b1 (h) | w2 (h) | b2] into FP64 parts.

    W1 is returned as [h, m] (row j = weights of hidden unit j).
    """
    w = np.asarray(w, dtype=np.float64)
    W1 = w[: m * h].reshape(m, h).T
    b1 = w[m * h: m * h + h]
    w2 = w[m * h + h: m * h + 2 * h]
    b2 = w[m * h + 2 * h]
    return W1, b1, w2, b2


def mlp_forward(w: np.ndarray, q_s: np.ndarray, m: int, h: int) -> np.ndarray:
    """Filter prediction d^f(q) = w2 . ReLU(W1 q + b1) + b2, FP64, for each query row."""
    W1, b1, w2, b2 = unpack_mlp(w, m, h)
    z = q_s.astype(np.float64) @ W1.T + b1
    return np.maximum(z, 0.0) @ w2 + b2


def mlp_mse_grad(w: np.ndarray, X: np.ndarray, y: np.ndarray, m: int, h: int):
    """Loss mean((d^f - y)^2) over a batch and its gradient in the packed layout, FP64."""
    W1, b1, w2, b2 = unpack_mlp(w, m, h)
    X = X.astype(np.float64)
    z = X @ W1.T + b1                       # [B, h]
    a = np.maximum(z, 0.0)
    yhat = a @ w2 + b2
    r = yhat - y
    B = X.shape[0]
    loss = float((r ** 2).mean())
    g = 2.0 * r / B                         # dL/dyhat
    gw2 = a.T @ g
    gb2 = g.sum()
    delta = np.outer(g, w2) * (z > 0)       # [B, h]
    gW1 = delta.T @ X                       # [h, m]
    gb1 = delta.sum(axis=0)
    grad = np.empty(m * h + 2 * h + 1)
    grad[: m * h] = gW1.T.reshape(-1)       # back to input-major
    grad[m * h: m * h + h] = gb1
    grad[m * h + h: m * h + 2 * h] = gw2
    grad[-1] = gb2
    return loss, grad


# ---------------------------------------------------------------------------
# Learned filter: two-layer 1-D CNN (Section "Varying Model Type": two
# convolutional layers, kernel size 3, latent channels equal to the series
# length).  Readings where the paper is silent: both layers are
# cross-correlations over the series positions with one zero of padding at
# each end (output length = input length), each followed by ReLU, and the
# prediction is a linear readout of the second layer's channels averaged over
# the positions.
# ---------------------------------------------------------------------------

def cnn_param_count(C: int) -> int:
    """Floats of a packed CNN filter with C channels:
    [W1 (C, 3) | b1 (C) | W2 (C_out, C_in, 3) | b2 (C) | w3 (C) | b3]."""
    return 3 * C + C + 3 * C * C + C + C + 1


def unpack_cnn(w: np.ndarray, C: int):
    w = np.asarray(w, dtype=np.float64)
    o = 0
    W1 = w[o: o + 3 * C].reshape(C, 3); o += 3 * C
    b1 = w[o: o + C]; o += C
    W2 = w[o: o + 3 * C * C].reshape(C, C, 3); o += 3 * C * C
    b2 = w[o: o + C]; o += C
    w3 = w[o: o + C]; o += C
    b3 = w[o]
    return W1, b1, W2, b2, w3, b3


def _cnn_layers(w, X, C):
    """Pre-activations z1 [B, C, m], z2 [B, C, m] for query rows X [B, m]."""
    W1, b1, W2, b2, w3, b3 = unpack_cnn(w, C)
    X = np.asarray(X, dtype=np.float64)
    B, m = X.shape
    xp = np.zeros((B, m + 2))
    xp[:, 1:m + 1] = X
    # tap t reads position p + t - 1
    z1 = b1[None, :, None] + sum(W1[None, :, t, None] * xp[:, None, t:t + m] for t in range(3))
    h1 = np.maximum(z1, 0.0)
    hp = np.zeros((B, C, m + 2))
    hp[:, :, 1:m + 1] = h1
    z2 = b2[None, :, None] + sum(np.einsum("oc,bcp->bop", W2[:, :, t], hp[:, :, t:t + m]) for t in range(3))
    return z1, h1, hp, z2


def cnn_forward(w: np.ndarray, q_s: np.ndarray, C: int) -> np.ndarray:
    """CNN filter prediction d^f(q) = b3 + sum_c w3[c] mean_p ReLU(z2[c, p]),
    FP64, for each query row (the series are the single input channel)."""
    W1, b1, W2, b2, w3, b3 = unpack_cnn(w, C)
    _, _, _, z2 = _cnn_layers(w, q_s, C)
    return np.maximum(z2, 0.0).mean(axis=2) @ w3 + b3


def cnn_mse_grad(w: np.ndarray, X: np.ndarray, y: np.ndarray, C: int):
    """Loss mean((d^f - y)^2) over a batch and its gradient in the packed
    CNN layout, FP64 (backpropagation through the two correlations)."""
    W1, b1, W2, b2, w3, b3 = unpack_cnn(w, C)
    X = np.asarray(X, dtype=np.float64)
    B, m = X.shape
    z1, h1, hp, z2 = _cnn_layers(w, X, C)
    h2 = np.maximum(z2, 0.0)
    pooled = h2.mean(axis=2)                       # [B, C]
    r = pooled @ w3 + b3 - y
    loss = float((r ** 2).mean())
    g = 2.0 * r / B                                # dL/dprediction
    gw3 = pooled.T @ g
    gb3 = g.sum()
    d2 = (g[:, None, None] * w3[None, :, None] / m) * (z2 > 0)      # dL/dz2 [B, C, m]
    gb2 = d2.sum(axis=(0, 2))
    gW2 = np.stack([np.einsum("bop,bcp->oc", d2, hp[:, :, t:t + m]) for t in range(3)], axis=2)
    # dL/dh1[c, q] = sum_o sum_t W2[o, c, t] d2[o, q - t + 1]
    dhp = np.zeros((B, C, m + 2))
    for t in range(3):
        dhp[:, :, t:t + m] += np.einsum("oc,bop->bcp", W2[:, :, t], d2)
    d1 = dhp[:, :, 1:m + 1] * (z1 > 0)                                # dL/dz1
    gb1 = d1.sum(axis=(0, 2))
    xp = np.zeros((B, m + 2))
    xp[:, 1:m + 1] = X
    gW1 = np.stack([np.einsum("bcp,bp->c", d1, xp[:, t:t + m]) for t in range(3)], axis=1)
    grad = np.concatenate([gW1.reshape(-1), gb1, gW2.reshape(-1), gb2, gw3, [gb3]])
    return loss, grad


# ---------------------------------------------------------------------------
# Search (Algorithm 2) in a round schedule
# ---------------------------------------------------------------------------

@dataclass
class SearchResult:
    ids: np.ndarray        # [nq, k] int64, -1 when fewer than k
    dist: np.ndarray       # [nq, k] FP64 Euclidean
    scanned: np.ndarray    # [nq, N] bool: leaf searched
    lb_pruned: np.ndarray  # [nq, N] bool
    f_pruned: np.ndarray   # [nq, N] bool
    near_tie: np.ndarray   # [nq, N] bool: decision within rel_tie of tau


def leafi_search(lb, order, leaf_d, leaf_ids, k, has_filter=None, dF=None, schedule=(1,),
                 rel_tie: float = 1e-5) -> SearchResult:
    """LeaFi-enhanced search (Algorithm 2) for each query, in rounds.

    The best-so-far tau is +inf until k results are held, then the k-th best
    distance.  Leaves are taken in visit order; a leaf is pruned when
    d^lb > tau, or when it holds a filter and d^F > tau (d^F = d^f - o);
    otherwise it is searched and its members merged into the result.
    Round r takes the next schedule[r] leaves that survive (the last entry
    repeats; 0 means "all that survive"), deciding all of them with the tau
    from before the round.  schedule=(1,) is the paper's sequential loop.

    leaf_d / leaf_ids [nq, N, k] are the per-leaf exact top-k (searching a
    leaf yields exactly these).  dF [nq, N] holds d^f - o for leaves with a
    filter (+inf disables a filter).
    """
    nq, N = lb.shape
    if has_filter is None:
        has_filter = np.zeros(N, dtype=bool)
    ids = np.full((nq, k), -1, dtype=np.int64)
    dist = np.full((nq, k), np.inf)
    scanned = np.zeros((nq, N), dtype=bool)
    lbp = np.zeros((nq, N), dtype=bool)
    fp = np.zeros((nq, N), dtype=bool)
    tie = np.zeros((nq, N), dtype=bool)
    kk = leaf_d.shape[2]
    for qi in range(nq):
        res_d = []            # list of (d, id)
        tau = math.inf
        pos = 0
        r = 0
        while pos < N:
            want = schedule[min(r, len(schedule) - 1)]
            take = []
            while pos < N and (want == 0 or len(take) < want):
                L = int(order[qi, pos])
                pos += 1
                if tau < math.inf:
                    tie[qi, L] = abs(lb[qi, L] - tau) <= rel_tie * tau or (
                        bool(has_filter[L]) and abs(dF[qi, L] - tau) <= rel_tie * tau)
                if lb[qi, L] > tau:
                    lbp[qi, L] = True
                    continue
                if has_filter[L] and dF[qi, L] > tau:
                    fp[qi, L] = True
                    continue
                take.append(L)
            for L in take:
                scanned[qi, L] = True
                for j in range(min(k, kk)):
                    if leaf_ids[qi, L, j] < 0:
                        break
                    res_d.append((leaf_d[qi, L, j], int(leaf_ids[qi, L, j])))
            res_d.sort()
            res_d = res_d[:k]
            if len(res_d) == k:
                tau = res_d[-1][0]
            r += 1
        for j, (d, i) in enumerate(res_d):
            ids[qi, j] = i
            dist[qi, j] = d
    return SearchResult(ids, dist, scanned, lbp, fp, tie)


def bsf_before(leaf_d: np.ndarray, order: np.ndarray, k: int) -> np.ndarray:
    """d^bsf(c, i): the k-th smallest distance over all series in the leaves that
    precede leaf i in c's visit order (+inf while fewer than k series precede).

    This is the best-so-far of the exact search just before it visits leaf i
    (Algorithm 1's global training targets T_g pair each d^L with it).
    Returns [nq, N] indexed by leaf id.
    """
    nq, N, kk = leaf_d.shape
    out = np.empty((nq, N))
    for c in range(nq):
        pool = np.full(k, np.inf)
        for pos in range(N):
            L = order[c, pos]
            out[c, L] = pool[k - 1]
            pool = np.sort(np.concatenate([pool, leaf_d[c, L, :k]]))[:k]
    return out


# ---------------------------------------------------------------------------
# Conformal auto-tuning (Section "Filter Conformal Auto-tuning", Algorithm 4)
# ---------------------------------------------------------------------------

def simulated_recall(dfilt, dbsf, nbr_leaf, has_filter, offsets) -> float:
    """Recall of the simulated search on the calibration queries for one offset vector.

    A true neighbour of query c that lives in leaf i is kept unless leaf i has
    a filter and d^f(c, i) - o_i > d^bsf(c, i).  Recall is the mean over
    queries of (kept neighbours / k).
    dfilt, dbsf [nc, N]; nbr_leaf [nc, k] leaf of each true neighbour.
    """
    nc, k = nbr_leaf.shape
    rows = np.repeat(np.arange(nc), k)
    leaf = nbr_leaf.reshape(-1)
    pruned = has_filter[leaf] & (dfilt[rows, leaf] - offsets[leaf] > dbsf[rows, leaf])
    kept = int((~pruned).sum())
    return kept / (nc * k)


def abs_errors(dfilt: np.ndarray, dL: np.ndarray) -> np.ndarray:
    """Non-conformity scores alpha = |d^f - d^L| on the calibration set, [nc, N]."""
    return np.abs(dfilt - dL)


def autotune_curve(dfilt, dL, dbsf, nbr_leaf, has_filter):
    """Algorithm 4: for each sorted position j the offsets o_i = alpha_{i,(j)} and
    the simulated recall q_j.

    Returns (offsets [nc + 1, N], q [nc + 1]); row nc (the appended last
    position) has o = +inf (filters never prune) and q = 1.  Leaves without a
    filter carry +inf throughout.
    """
    nc, N = dfilt.shape
    alpha = np.sort(abs_errors(dfilt, dL), axis=0)   # ascending per filter
    offs = np.full((nc + 1, N), np.inf)
    offs[:nc, has_filter] = alpha[:, has_filter]
    q = np.empty(nc + 1)
    for j in range(nc):
        q[j] = simulated_recall(dfilt, dbsf, nbr_leaf, has_filter, offs[j])
    q[nc] = 1.0
    return offs, q


def conformal_target(target: float, nc: int, corrected: bool = True) -> float:
    """Finite-sample corrected level min(1, ceil((nc + 1) * target) / nc)."""
    if not corrected:
        return target
    return min(1.0, math.ceil((nc + 1) * target - 1e-9) / nc)


def step_offsets(offs, q, target, nc, corrected=True):
    """Step mapping from a recall target to offsets: the first position j whose
    (suffix-minimum) recall reaches the corrected target."""
    qhat = np.minimum.accumulate(q[::-1])[::-1]
    t = conformal_target(target, nc, corrected)
    j = int(np.argmax(qhat >= t - 1e-12))
    return j, offs[j]


def steffen_fit(x: np.ndarray, y: np.ndarray):
    """Steffen (1990) monotone cubic interpolant through (x_i, y_i), x strictly increasing.

    Returns the per-interval cubic coefficients (a, b, c, d) with
    y(t) = a (t - x_i)^3 + b (t - x_i)^2 + c (t - x_i) + d on [x_i, x_{i+1}].
    Slopes: interior y'_i = (sign(s_{i-1}) + sign(s_i)) * min(|s_{i-1}|, |s_i|,
    |p_i| / 2) with p_i the slope of the parabola through the three points;
    end slopes from the one-sided parabola, limited the same way.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = len(x)
    if n == 1:
        return x, np.zeros((1, 4)) + np.array([0, 0, 0, y[0]])
    h = np.diff(x)
    s = np.diff(y) / h
    yp = np.zeros(n)
    if n == 2:
        yp[:] = s[0]
    else:
        for i in range(1, n - 1):
            p = (s[i - 1] * h[i] + s[i] * h[i - 1]) / (h[i - 1] + h[i])
            yp[i] = (np.sign(s[i - 1]) + np.sign(s[i])) * min(abs(s[i - 1]), abs(s[i]), 0.5 * abs(p))
        p0 = s[0] * (1 + h[0] / (h[0] + h[1])) - s[1] * h[0] / (h[0] + h[1])
        yp[0] = 2 * s[0] if (p0 * s[0] > 0 and abs(p0) > 2 * abs(s[0])) else (p0 if p0 * s[0] > 0 else 0.0)
        pn = s[-1] * (1 + h[-1] / (h[-1] + h[-2])) - s[-2] * h[-1] / (h[-1] + h[-2])
        yp[-1] = 2 * s[-1] if (pn * s[-1] > 0 and abs(pn) > 2 * abs(s[-1])) else (pn if pn * s[-1] > 0 else 0.0)
    coef = np.zeros((n - 1, 4))
    for i in range(n - 1):
        coef[i, 0] = (yp[i] + yp[i + 1] - 2 * s[i]) / h[i] ** 2
        coef[i, 1] = (3 * s[i] - 2 * yp[i] - yp[i + 1]) / h[i]
        coef[i, 2] = yp[i]
        coef[i, 3] = y[i]
    return x, coef


def steffen_eval(fit, t: float) -> float:
    x, coef = fit
    if len(x) == 1 or t <= x[0]:
        return float(coef[0, 3]) if t <= x[0] else float(coef[0, 3])
    if t >= x[-1]:
        i = len(x) - 2
        dx = x[-1] - x[i]
    else:
        i = int(np.searchsorted(x, t, side="right") - 1)
        dx = t - x[i]
    a, b, c, d = coef[i]
    return float(((a * dx + b) * dx + c) * dx + d)


def steffen_offsets(offs, q, target, nc, corrected=True):
    """Paper variant of the mapping: per filter, Steffen's monotone interpolant of
    offset against recall through the points (q_j, o_{i,(j)}).  Equal recalls
    keep the largest offset; a target above the largest finite-offset recall
    turns the filter off (+inf); below the smallest it takes the first offset.
    """
    t = conformal_target(target, nc, corrected)
    N = offs.shape[1]
    out = np.full(N, np.inf)
    for i in range(N):
        col = offs[:, i]
        ok = np.isfinite(col)
        if not ok.any():
            continue
        xs, ys = q[ok], col[ok]
        ux = np.unique(xs)
        uy = np.array([ys[xs == v].max() for v in ux])
        if t > ux[-1]:
            continue
        if t <= ux[0]:
            out[i] = uy[0]
            continue
        out[i] = steffen_eval(steffen_fit(ux, uy), t)
    return out


# ---------------------------------------------------------------------------
# Leaf selection (Algorithm 3, Equation 4)
# ---------------------------------------------------------------------------

def size_threshold(a: float, tF: float, tS: float) -> float:
    """th = a * t^F / t^S: a leaf is worth a filter if searching it costs more than
    a filter inference divided by the filter pruning probability 1/a."""
    return a * tF / tS


def select_leaves(sizes, th: float, w: float, cM: float) -> np.ndarray:
    """Greedy selection: leaves by size, largest first (ties: smaller leaf id);
    take a leaf when its size is >= th and its filter still fits in memory
    (w_used + w <= c^M).  Returns selected leaf ids in selection order."""
    sizes = np.asarray(sizes)
    o = np.lexsort((np.arange(len(sizes)), -sizes))
    used = 0.0
    sel = []
    for L in o:
        if sizes[L] >= th and used + w <= cM:
            sel.append(int(L))
            used += w
    return np.array(sel, dtype=np.int64)


# ---------------------------------------------------------------------------
# Leaf selection as a knapsack (Section "Leaf Node Selection", Equations 1-2)
# ---------------------------------------------------------------------------

def knapsack_01(values, weights, capacity: int) -> np.ndarray:
    """Equation 1: the 0/1 knapsack, maximise sum v_i x_i subject to
    sum w_i x_i <= capacity, solved exactly by dynamic programming over the
    (non-negative integer) weights.  best[c] after item i is the largest value
    of a subset of items 0..i of weight <= c; the chosen subset is read back
    from the table.  Returns the chosen item indices, ascending."""
    v = np.asarray(values, dtype=np.float64)
    wt = np.asarray(weights, dtype=np.int64)
    n = len(v)
    C = int(capacity)
    if n == 0 or C < 0:
        return np.zeros(0, dtype=np.int64)
    best = np.zeros((n + 1, C + 1))
    for i in range(n):
        best[i + 1] = best[i]
        if wt[i] <= C:
            cand = best[i, : C + 1 - wt[i]] + v[i]
            best[i + 1, wt[i]:] = np.maximum(best[i, wt[i]:], cand)
    chosen = []
    c = C
    for i in range(n - 1, -1, -1):
        if best[i + 1, c] != best[i, c]:  # item i is needed for this optimum
            chosen.append(i)
            c -= wt[i]
    return np.array(sorted(chosen), dtype=np.int64)


def selection_estimates(lb: np.ndarray, leaf_d1: np.ndarray, order: np.ndarray):
    """Per-leaf pruning probabilities for Equation 2, estimated on training
    queries by following the exact 1-NN search (no filters) in visit order.

    Reading (the paper leaves the estimator open): with d^bsf the best
    distance over the leaves ahead of leaf i in the query's visit order,
    p^lb_i is the share of queries whose bound prunes leaf i (d^lb > d^bsf),
    and the ideal filter rate p^F*_i is the share of the remaining visits in
    which leaf i holds nothing closer than d^bsf (d^L > d^bsf), i.e. what a
    filter that predicts d^L exactly would prune (0 when no query reaches the
    leaf).  lb, leaf_d1 [nq, N] by leaf id (leaf_d1 = node-wise 1-NN
    distance d^L); order [nq, N].  Returns (p_lb, p_f_ideal), each [N]."""
    nq, N = lb.shape
    dbsf = bsf_before(leaf_d1[:, :, None], order, 1)
    pruned = lb > dbsf
    reached = ~pruned
    ideal = reached & (leaf_d1 > dbsf)
    p_lb = pruned.sum(axis=0) / nq
    n_reach = reached.sum(axis=0)
    p_f = np.where(n_reach > 0, ideal.sum(axis=0) / np.maximum(n_reach, 1), 0.0)
    return p_lb, p_f


def leaf_benefit(sizes, p_lb, p_f, tS: float, tF: float) -> np.ndarray:
    """Equation 2: the expected search time a filter saves on leaf i,
    b_i = (1 - p^lb_i) (p^F_i t^S |N_i| - t^F)."""
    sizes = np.asarray(sizes, dtype=np.float64)
    return (1.0 - np.asarray(p_lb, dtype=np.float64)) * (np.asarray(p_f, dtype=np.float64) * tS * sizes - tF)


def select_knapsack(sizes, p_lb, p_f_ideal, a: float, tS: float, tF: float, w: int, cM: int):
    """Leaf selection by Equations 1-2 with per-leaf estimates: p^F_i is the
    ideal rate discounted by the hyperparameter a (p^F_i = p^F*_i / a, which
    is Algorithm 3's p^F = 1 / a when every leaf's ideal rate is 1); leaves
    with b_i <= 0 are never taken (they would slow the search); the rest go
    into the knapsack of capacity c^M with weight w bytes per filter (one
    architecture for all filters, so the weights are equal).  Returns
    (selected leaf ids ordered by benefit, largest first, ties by leaf id;
    b [N])."""
    b = leaf_benefit(sizes, p_lb, np.asarray(p_f_ideal, dtype=np.float64) / a, tS, tF)
    cand = np.flatnonzero(b > 0)
    # equal weights: sum w x <= c^M is "at most floor(c^M / w) filters", so
    # each filter weighs one unit (capacity beyond the candidates is unused)
    cap = min(int(cM) // int(w), len(cand)) if w > 0 else len(cand)
    chosen = cand[knapsack_01(b[cand], np.ones(len(cand), dtype=np.int64), cap)]
    o = np.lexsort((chosen, -b[chosen]))
    return chosen[o].astype(np.int64), b


# ---------------------------------------------------------------------------
# Quality measure (Section "Evaluation Setup", evaluation measures)
# ---------------------------------------------------------------------------

def recall_at_k(ret_ids: np.ndarray, ret_d64: np.ndarray, true_d: np.ndarray, rel: float = 1e-12) -> np.ndarray:
    """recall@k per query: returned items whose exact distance is within the k-th
    exact distance (ties with the k-th count as hits), divided by k."""
    k = true_d.shape[1]
    kth = true_d[:, k - 1:k]
    hit = (ret_ids >= 0) & (ret_d64 <= kth * (1 + rel))
    return hit.sum(axis=1) / k
