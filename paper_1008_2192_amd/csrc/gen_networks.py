"""Generator of straight-line min/max median networks for the HIP kernels.

Emits ``medtile.inc``: device functions that compute a k x k median filter for a
small register tile of outputs (ty x tx) from a (ty+k-1) x (tx+k-1) input patch,
plus the 25-element sort used by the masked replacement.

Construction (a separable, shared sorting-network selection):
  * every window is a union of column segments; a tile of windows is handled by
    recursive halving of the tile.  The inputs common to every window of a
    sub-tile are kept as one sorted list, and each half adds the inputs it shares
    (a rectangle, sorted once and memoised) by a merge;
  * after each merge the list is pruned by rank: for windows of k*k elements with
    target rank m = (k*k-1)/2, an element at position p of the sorted common set C
    can be the median of some window only if m - (k*k-|C|) <= p <= m.  Elements
    below that range are below every window's median (the target rank drops by
    their number), elements above it are above (the rank is unchanged);
  * a final dead-code pass keeps only the min/max operations that reach an output.
Sorted rectangles are built from sorted column segments by pairwise odd-even
merges (Batcher), merges are pruned to the output positions still needed, and
correctness is checked here with the 0-1 principle on random and exhaustive
0/1 inputs (any min/max network that selects rank m correctly on every 0/1 input
does so on every input).

Run as a script to write ``medtile.inc`` next to this file.
"""
from __future__ import annotations

import itertools
import os
import random
import sys
from typing import Dict, List, Sequence, Tuple


# ---------------------------------------------------------------------------
# symbolic network
# ---------------------------------------------------------------------------

class Net:
    """SSA list of ops; values 0..n_in-1 are inputs."""

    def __init__(self, n_in: int):
        self.n_in = n_in
        self.ops: List[Tuple[str, int, int]] = []     # (kind, a, b) -> value id n_in + i

    def _new(self, kind, a, b):
        self.ops.append((kind, a, b))
        return self.n_in + len(self.ops) - 1

    def cmpx(self, a: int, b: int) -> Tuple[int, int]:
        if a == b:
            return a, b
        return self._new("min", a, b), self._new("max", a, b)

    # -- sorting and merging --------------------------------------------------
    def sort(self, vals: Sequence[int]) -> List[int]:
        v = list(vals)
        n = len(v)
        for i, j in batcher_pairs(n):
            v[i], v[j] = self.cmpx(v[i], v[j])
        return v

    def merge(self, a: Sequence[int], b: Sequence[int]) -> List[int]:
        """Odd-even merge of two sorted lists of arbitrary lengths."""
        a, b = list(a), list(b)
        if not a:
            return b
        if not b:
            return a
        if len(a) == 1 and len(b) == 1:
            lo, hi = self.cmpx(a[0], b[0])
            return [lo, hi]
        n = len(a) + len(b)
        # sort the concatenation with a network that knows both halves are sorted:
        # Batcher's merge-exchange pass restricted to the final merge levels is
        # awkward for unequal sizes, so use the recursive odd-even merge.
        ev = self.merge(a[0::2], b[0::2])
        od = self.merge(a[1::2], b[1::2])
        out = [None] * n
        # interleave: ev gives candidates for positions 0,2,4..; od for 1,3,5..
        # then compare-exchange neighbours (2i-1, 2i)
        seq = []
        ie, io = 0, 0
        # standard recombination for the odd-even merge with arbitrary sizes:
        # result = ev[0], then pairs (od[i], ev[i+1]) compare-exchanged, then tail
        seq.append(ev[0])
        i = 0
        while i < len(od) or i + 1 < len(ev):
            x = od[i] if i < len(od) else None
            y = ev[i + 1] if i + 1 < len(ev) else None
            if x is not None and y is not None:
                lo, hi = self.cmpx(x, y)
                seq += [lo, hi]
            elif x is not None:
                seq.append(x)
            else:
                seq.append(y)
            i += 1
        assert len(seq) == n
        return seq


def batcher_pairs(n: int) -> List[Tuple[int, int]]:
    """Batcher's merge-exchange sorting network for any n (Knuth, TAOCP 5.2.2 M)."""
    pairs = []
    if n < 2:
        return pairs
    t = (n - 1).bit_length()
    p = 1 << (t - 1)
    while p > 0:
        q = 1 << (t - 1)
        r = 0
        d = p
        while True:
            for i in range(n - d):
                if (i & p) == r:
                    pairs.append((i, i + d))
            if q == p:
                break
            d = q - p
            q >>= 1
            r = p
        p >>= 1
    return pairs


# ---------------------------------------------------------------------------
# rank-pruned tile median
# ---------------------------------------------------------------------------

class TileMedian:
    """k x k median for a ty x tx tile of outputs; input patch (ty+k-1) x (tx+k-1)."""

    def __init__(self, k: int, ty: int, tx: int):
        self.k, self.ty, self.tx = k, ty, tx
        self.ph, self.pw = ty + k - 1, tx + k - 1
        self.net = Net(self.ph * self.pw)
        self.memo: Dict[Tuple[int, int, int, int], List[int]] = {}
        self.outputs: Dict[Tuple[int, int], int] = {}
        self.m = (k * k - 1) // 2

    def inp(self, r, c):
        return r * self.pw + c

    def sorted_rect(self, r0, r1, c0, c1) -> List[int]:
        """Sorted list of patch inputs rows [r0,r1) x cols [c0,c1) (memoised)."""
        key = (r0, r1, c0, c1)
        if key in self.memo:
            return self.memo[key]
        nr, nc = r1 - r0, c1 - c0
        if nr <= 0 or nc <= 0:
            res = []
        elif nc == 1:
            if nr <= 2:
                res = self.net.sort([self.inp(r, c0) for r in range(r0, r1)])
            else:
                # split the column segment to share pieces between overlapping windows
                h = nr // 2
                res = self.net.merge(self.sorted_rect(r0, r0 + h, c0, c1),
                                     self.sorted_rect(r0 + h, r1, c0, c1))
        else:
            h = nc // 2
            res = self.net.merge(self.sorted_rect(r0, r1, c0, c0 + h),
                                 self.sorted_rect(r0, r1, c0 + h, c1))
        self.memo[key] = res
        return res

    def common(self, y0, y1, x0, x1):
        """Rectangle of patch inputs shared by the windows of outputs rows [y0,y1),
        cols [x0,x1) (output (i,j) covers patch rows i..i+k-1, cols j..j+k-1)."""
        k = self.k
        return (y1 - 1, y0 + k, x1 - 1, x0 + k)

    def build(self):
        k = self.k
        kk = k * k
        # root: the whole tile
        self._node(0, self.ty, 0, self.tx, [], self.m, None)
        return self

    def _node(self, y0, y1, x0, x1, L, rank, prev_rect):
        k = self.k
        kk = k * k
        r0, r1, c0, c1 = self.common(y0, y1, x0, x1)
        cur = (max(r0, 0), r1, max(c0, 0), c1)
        size_c = max(0, r1 - r0) * max(0, c1 - c0)
        # new elements D = cur \ prev (a rectangle difference)
        D_lists = []
        if prev_rect is None:
            if size_c > 0:
                D_lists.append(self.sorted_rect(r0, r1, c0, c1))
        else:
            pr0, pr1, pc0, pc1 = prev_rect
            if size_c > 0:
                if pr1 - pr0 <= 0 or pc1 - pc0 <= 0:
                    D_lists.append(self.sorted_rect(r0, r1, c0, c1))
                else:
                    # cur contains prev; difference = up to 4 bands
                    assert r0 <= pr0 and pr1 <= r1 and c0 <= pc0 and pc1 <= c1
                    if r0 < pr0:
                        D_lists.append(self.sorted_rect(r0, pr0, c0, c1))
                    if pr1 < r1:
                        D_lists.append(self.sorted_rect(pr1, r1, c0, c1))
                    if c0 < pc0:
                        D_lists.append(self.sorted_rect(pr0, pr1, c0, pc0))
                    if pc1 < c1:
                        D_lists.append(self.sorted_rect(pr0, pr1, pc1, c1))
        # merge: combine D pieces, then with L, pruning to the needed window
        e = kk - size_c                  # elements of each window not yet in the list
        lo_need = max(0, rank - e)
        hi_need = rank
        lst = L
        for D in D_lists:
            lst, shift = self._pruned_merge(lst, D, lo_need, hi_need)
            lo_need -= shift
            hi_need -= shift
            rank -= shift
        # prune by rank
        drop_lo = max(0, rank - e)
        lst = lst[drop_lo:rank + 1]
        rank -= drop_lo
        if y1 - y0 == 1 and x1 - x0 == 1:
            assert e == 0 and len(lst) == 1 and rank == 0, (e, len(lst), rank)
            self.outputs[(y0, x0)] = lst[0]
            return
        rect = (r0, r1, c0, c1) if size_c > 0 else (0, 0, 0, 0)
        # split the longer side (rows first on ties: columns are sorted vertically)
        if (y1 - y0) >= (x1 - x0):
            ym = (y0 + y1) // 2
            self._node(y0, ym, x0, x1, lst, rank, rect)
            self._node(ym, y1, x0, x1, lst, rank, rect)
        else:
            xm = (x0 + x1) // 2
            self._node(y0, y1, x0, xm, lst, rank, rect)
            self._node(y0, y1, xm, x1, lst, rank, rect)

    def _pruned_merge(self, A, B, lo, hi):
        """Merge sorted A and B keeping output positions [lo, hi] (others may be
        dropped).  Returns (list, shift) where list[i] is the element of merged
        position i + shift for positions kept."""
        a, b = len(A), len(B)
        # drop elements that can only land above hi
        A2, B2 = A[:hi + 1], B[:hi + 1]
        # drop elements that can only land below lo
        dA = max(0, lo - len(B2))
        dB = max(0, lo - len(A2))
        A2, B2 = A2[dA:], B2[dB:]
        merged = self.net.merge(A2, B2)
        return merged, dA + dB


# ---------------------------------------------------------------------------
# dead-code elimination and op counting
# ---------------------------------------------------------------------------

def live_ops(net: Net, outs: Sequence[int]) -> List[bool]:
    live = [False] * len(net.ops)
    stack = [o for o in outs if o >= net.n_in]
    seen = set()
    while stack:
        v = stack.pop()
        if v in seen or v < net.n_in:
            continue
        seen.add(v)
        i = v - net.n_in
        live[i] = True
        _, a, b = net.ops[i]
        stack += [a, b]
    return live


def count_ops(net: Net, outs) -> int:
    return sum(live_ops(net, outs))


def fused_count(net: Net, outs) -> int:
    """Estimate after min3/max3 fusion: a min (max) whose single use is another min
    (max) folds into it."""
    live = live_ops(net, outs)
    uses = {}
    for i, (kind, a, b) in enumerate(net.ops):
        if not live[i]:
            continue
        for x in (a, b):
            uses.setdefault(x, []).append(i)
    folded = 0
    for i, (kind, a, b) in enumerate(net.ops):
        if not live[i]:
            continue
        v = net.n_in + i
        u = uses.get(v, [])
        if len(u) == 1 and net.ops[u[0]][0] == kind and v not in outs:
            folded += 1
    return sum(live) - folded


def evaluate(net: Net, inputs, outs):
    vals = list(inputs) + [None] * len(net.ops)
    live = live_ops(net, outs)
    n = net.n_in
    for i, (kind, a, b) in enumerate(net.ops):
        if not live[i]:
            continue
        x, y = vals[a], vals[b]
        vals[n + i] = (min(x, y) if kind == "min" else max(x, y))
    return [vals[o] for o in outs]


def evaluate_np(net: Net, inputs, outs):
    import numpy as np
    vals = list(inputs) + [None] * len(net.ops)
    live = live_ops(net, outs)
    n = net.n_in
    for i, (kind, a, b) in enumerate(net.ops):
        if not live[i]:
            continue
        vals[n + i] = np.minimum(vals[a], vals[b]) if kind == "min" else np.maximum(vals[a], vals[b])
    return [vals[o] for o in outs]


def check_tile(tm: TileMedian, trials=2000, seed=0):
    import numpy as np
    rng = np.random.default_rng(seed)
    k, ty, tx = tm.k, tm.ty, tm.tx
    outs = [tm.outputs[(i, j)] for i in range(ty) for j in range(tx)]
    # random 0/1 inputs (biased densities to hit the median boundary) and random ties
    for mode in ("01", "ties"):
        if mode == "01":
            p = rng.random((trials, 1))
            X = (rng.random((trials, tm.ph * tm.pw)) < p).astype(np.int8)
        else:
            X = rng.integers(0, 4, (trials, tm.ph * tm.pw)).astype(np.int8)
        got = evaluate_np(tm.net, [X[:, i] for i in range(X.shape[1])], outs)
        P = X.reshape(trials, tm.ph, tm.pw)
        for idx, (i, j) in enumerate([(i, j) for i in range(ty) for j in range(tx)]):
            win = P[:, i:i + k, j:j + k].reshape(trials, -1)
            exp = np.sort(win, axis=1)[:, tm.m]
            assert (got[idx] == exp).all(), (k, ty, tx, i, j, mode)
    return True


# ---------------------------------------------------------------------------
# emission
# ---------------------------------------------------------------------------

def _ref(net: Net, x: int) -> str:
    return f"v[{x}]" if x < net.n_in else f"t{x}"


def dfs_order(net: Net, outs: Sequence[int]) -> List[int]:
    """Op indices in depth-first post-order from the outputs: each value is computed
    just before its first use, which keeps fewer values live at a time."""
    order, seen = [], set()
    for o in outs:
        stack = [(o, False)]
        while stack:
            v, done = stack.pop()
            if v < net.n_in or v in seen:
                continue
            if done:
                seen.add(v)
                order.append(v - net.n_in)
                continue
            stack.append((v, True))
            _, a, b = net.ops[v - net.n_in]
            stack.append((b, False))
            stack.append((a, False))
    return order


EMIT_ORDER = os.environ.get("CRB_NET_ORDER", "seq")


def emit_tile_function(name: str, tm: TileMedian) -> str:
    net = tm.net
    outs = [tm.outputs[(i, j)] for i in range(tm.ty) for j in range(tm.tx)]
    live = live_ops(net, outs)
    nops = sum(live)
    lines = [f"// {tm.k}x{tm.k} median of a {tm.ty}x{tm.tx} output tile from a "
             f"{tm.ph}x{tm.pw} patch (row-major); {nops} min/max ops "
             f"({nops / (tm.ty * tm.tx):.1f} per output)",
             f"template <typename T>",
             f"__device__ __forceinline__ void {name}(const T (&v)[{tm.ph * tm.pw}], "
             f"T (&o)[{tm.ty * tm.tx}]) {{"]
    order = dfs_order(net, outs) if EMIT_ORDER == "dfs" else [i for i in range(len(net.ops))
                                                                if live[i]]
    for i in order:
        kind, a, b = net.ops[i]
        fn = "vmin" if kind == "min" else "vmax"
        lines.append(f"  const T t{net.n_in + i} = {fn}({_ref(net, a)}, {_ref(net, b)});")
    for idx, o in enumerate(outs):
        lines.append(f"  o[{idx}] = {_ref(net, o)};")
    lines.append("}")
    return "\n".join(lines)


def emit_sort_function(name: str, n: int) -> str:
    pairs = batcher_pairs(n)
    lines = [f"// ascending sort of {n} values in place: Batcher merge-exchange, "
             f"{len(pairs)} compare-exchanges",
             "template <typename T>",
             f"__device__ __forceinline__ void {name}(T (&v)[{n}]) {{"]
    for i, j in pairs:
        lines.append(f"  {{ const T a = v[{i}], b = v[{j}]; v[{i}] = vmin(a, b); "
                     f"v[{j}] = vmax(a, b); }}")
    lines.append("}")
    return "\n".join(lines)


# tile shapes used by the kernels: (function name, k, ty, tx)
TILES = [("med5_t2x2", 5, 2, 2), ("med5_t1x2", 5, 1, 2), ("med5_t1x1", 5, 1, 1),
         ("med7_t1x1", 7, 1, 1)]


def generate(path: str, verify: bool = True) -> None:
    parts = ["// Generated by gen_networks.py -- do not edit.",
             "// Straight-line min/max median networks for the L.A.Cosmic kernels.",
             "// vmin/vmax must be defined for float and double before inclusion.",
             "#pragma once", ""]
    for name, k, ty, tx in TILES:
        tm = TileMedian(k, ty, tx).build()
        if verify:
            check_tile(tm, trials=4000)
        parts.append(emit_tile_function(name, tm))
        parts.append("")
    parts.append(emit_sort_function("sort25", 25))
    parts.append("")
    text = "\n".join(parts)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write(text)
    os.replace(tmp, path)


def verify_sort(n: int) -> bool:
    """0-1 principle: the network sorts every 0/1 vector of length n."""
    import numpy as np
    pairs = batcher_pairs(n)
    X = ((np.arange(1 << n)[:, None] >> np.arange(n)[None, :]) & 1).astype(np.int8)
    for i, j in pairs:
        a, b = X[:, i].copy(), X[:, j].copy()
        X[:, i] = np.minimum(a, b)
        X[:, j] = np.maximum(a, b)
    return bool((np.diff(X, axis=1) >= 0).all())


if __name__ == "__main__" and (len(sys.argv) == 1 or sys.argv[1] != "count"):
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(
        os.path.abspath(__file__)), "medtile.inc")
    generate(out)
    print("wrote", out)


if __name__ == "__main__" and len(sys.argv) > 1 and sys.argv[1] == "count":
    for k, shapes in [(3, [(1, 1), (1, 4), (2, 4), (1, 8)]),
                      (5, [(1, 1), (1, 2), (2, 2), (2, 4), (4, 4), (1, 8), (2, 8), (4, 2), (8, 2)]),
                      (7, [(1, 1), (2, 2), (2, 4), (4, 2), (4, 4), (8, 2), (2, 8), (8, 4), (4, 8)])]:
        for ty, tx in shapes:
            tm = TileMedian(k, ty, tx).build()
            outs = list(tm.outputs.values())
            c = count_ops(tm.net, outs)
            f = fused_count(tm.net, outs)
            print(f"k={k} tile {ty}x{tx}: ops/px {c / (ty * tx):.1f}  fused {f / (ty * tx):.1f}")
