"""Host-side check of the scatter's addressing scheme (no GPU): an emulation of the
one-thread-per-block-record rule on small tile grids must write every CSR value
exactly once, at the (row, column) the CSR structure assigns to it, with the
owning record summing exactly the records that hold the same global pair."""
import numpy as np
import pytest

import workloads as W


def _overlap(i, j, p, e):
    lo_i, hi_i = max(0, i - p), min(e - 1, i)
    lo_j, hi_j = max(0, j - p), min(e - 1, j)
    return max(lo_i, lo_j) <= min(hi_i, hi_j)


def _dir_tables(n, p, T):
    e = n - p
    NG = T * (n - 1) + 1
    nb = [set() for _ in range(NG)]
    for t in range(T):
        for i in range(n):
            for j in range(n):
                if _overlap(i, j, p, e):
                    nb[t * (n - 1) + i].add(t * (n - 1) + j)
    lo = np.array([min(s) for s in nb])
    cnt = np.array([len(s) for s in nb])
    assert all(max(s) - min(s) + 1 == len(s) for s in nb)      # contiguous neighbour sets
    pre = np.concatenate([[0], np.cumsum(cnt)])
    return lo, cnt, pre


@pytest.mark.parametrize("name,kw", [("cfg1", {}), ("cfg3", {"n_el": 3}), ("cfg4", {"n_boxes": 3})])
def test_scatter_addressing(name, kw):
    import paper_2107_09568_amd as P
    w = W.make(name, **kw)
    plan = P.Plan.from_workload(w)
    rp, ci = plan.csr_host()
    pairs = plan.pairs()
    nT = [w.tile.ctrl.shape[2], w.tile.ctrl.shape[1], w.tile.ctrl.shape[0]]
    pT = list(w.tile.degree)
    tiles = list(w.tiles)
    D = [_dir_tables(nT[d], pT[d], tiles[d]) for d in range(3)]
    SX, SY = D[0][2][-1], D[1][2][-1]
    nnz = len(ci)
    hits = np.zeros(nnz, dtype=np.int64)
    row_of = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    lut = {(int(a), int(b)): k for k, (a, b) in enumerate(pairs)}
    owner_sum = {}
    for tile in range(plan.n_tiles):
        tt = [tile % tiles[0], (tile // tiles[0]) % tiles[1], tile // (tiles[0] * tiles[1])]
        for p, (A, B) in enumerate(pairs):
            ai = [A % nT[0], (A // nT[0]) % nT[1], A // (nT[0] * nT[1])]
            bi = [B % nT[0], (B // nT[0]) % nT[1], B // (nT[0] * nT[1])]
            if any(ai[d] == 0 and bi[d] == 0 and tt[d] > 0 for d in range(3)):
                continue
            up = [int(ai[d] == nT[d] - 1 and bi[d] == nT[d] - 1 and tt[d] < tiles[d] - 1) for d in range(3)]
            contrib = []
            for dz in range(up[2] + 1):
                for dy in range(up[1] + 1):
                    for dx in range(up[0] + 1):
                        t2 = tile + dx + tiles[0] * (dy + tiles[1] * dz)
                        A2 = A - dx * (nT[0] - 1) - nT[0] * (dy * (nT[1] - 1) + nT[1] * dz * (nT[2] - 1))
                        B2 = B - dx * (nT[0] - 1) - nT[0] * (dy * (nT[1] - 1) + nT[1] * dz * (nT[2] - 1))
                        contrib.append((t2, lut[(A2, B2)]))
            assert [c[0] for c in contrib] == sorted(c[0] for c in contrib)
            gA = [tt[d] * (nT[d] - 1) + ai[d] for d in range(3)]
            gB = [tt[d] * (nT[d] - 1) + bi[d] for d in range(3)]
            GA = gA[0] + D[0][0].size * (gA[1] + D[1][0].size * gA[2])
            GB = gB[0] + D[0][0].size * (gB[1] + D[1][0].size * gB[2])
            owner_sum[(GA, GB)] = contrib
            for (g, h, transpose) in ((gA, gB, False), (gB, gA, True)):
                if transpose and A == B:
                    continue
                c = [D[d][1][g[d]] for d in range(3)]
                base = 9 * (D[2][2][g[2]] * SY * SX + c[2] * (D[1][2][g[1]] * SX + c[1] * D[0][2][g[0]]))
                nnb = c[0] * c[1] * c[2]
                rank = ((h[2] - D[2][0][g[2]]) * c[1] + (h[1] - D[1][0][g[1]])) * c[0] + (h[0] - D[0][0][g[0]])
                G = g[0] + D[0][0].size * (g[1] + D[1][0].size * g[2])
                H = h[0] + D[0][0].size * (h[1] + D[1][0].size * h[2])
                for r in range(3):
                    for cc in range(3):
                        pos = base + 3 * r * nnb + 3 * rank + cc
                        hits[pos] += 1
                        assert row_of[pos] == 3 * G + r
                        assert ci[pos] == 3 * H + cc
    assert hits.min() == 1 and hits.max() == 1
    # the owner of a global pair sums every record that holds it
    count = {}
    for tile in range(plan.n_tiles):
        tt = [tile % tiles[0], (tile // tiles[0]) % tiles[1], tile // (tiles[0] * tiles[1])]
        for p, (A, B) in enumerate(pairs):
            ai = [A % nT[0], (A // nT[0]) % nT[1], A // (nT[0] * nT[1])]
            bi = [B % nT[0], (B // nT[0]) % nT[1], B // (nT[0] * nT[1])]
            gA = [tt[d] * (nT[d] - 1) + ai[d] for d in range(3)]
            gB = [tt[d] * (nT[d] - 1) + bi[d] for d in range(3)]
            GA = gA[0] + D[0][0].size * (gA[1] + D[1][0].size * gA[2])
            GB = gB[0] + D[0][0].size * (gB[1] + D[1][0].size * gB[2])
            count.setdefault((GA, GB), set()).add((tile, p))
    for key, recs in count.items():
        assert set(owner_sum[key]) == recs
