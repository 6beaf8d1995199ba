"""Host logic of the subdomain factor storage (CPU only): the tile envelope
the library reports is recomputed here from the subdomain node sets (owned
nodes plus `overlap` graph layers) and the library's own local order (its
local->global maps), and the envelope is shown to hold every nonzero of
the LU factors of a matrix with the subdomain's block pattern (elimination
without pivoting keeps its fill inside a nondecreasing profile)."""
import os

import numpy as np
import pytest
from scipy import sparse

import seird_inputs as si

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2208_01839_amd", "libseird.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libseird.so not built")

NC = 5


def node_graph(n, tri):
    r = np.concatenate([tri[:, 0], tri[:, 1], tri[:, 2], tri[:, 1], tri[:, 2], tri[:, 0]])
    c = np.concatenate([tri[:, 1], tri[:, 2], tri[:, 0], tri[:, 0], tri[:, 1], tri[:, 2]])
    G = sparse.csr_matrix((np.ones(len(r)), (r, c)), shape=(n, n))
    G.data[:] = 1.0
    return G


def subdomain_nodes(G, part, s, overlap):
    m = (part == s).astype(np.float64)
    for _ in range(overlap):
        m = np.minimum(1.0, m + G @ m)
    return np.nonzero(m)[0]


def envelope(G, order, tile):
    """lo (nondecreasing first tile column per tile row) and hi of the
    local matrix whose node k is order[k]."""
    nn = len(order)
    A = G[order][:, order].tocoo()
    left = np.arange(nn)
    np.minimum.at(left, A.row, A.col)
    nt = (NC * nn + tile - 1) // tile
    lo = np.arange(nt)
    for k in range(nn):
        for K in {(NC * k) // tile, (NC * k + NC - 1) // tile}:
            lo[K] = min(lo[K], (NC * left[k]) // tile)
    lo = np.minimum.accumulate(lo[::-1])[::-1]
    hi = np.array([max(K, int(np.nonzero(lo <= K)[0].max())) for K in range(nt)])
    return lo, hi


@pytest.mark.parametrize("tile", [32, 16])
def test_envelope_size_matches_library(tile):
    import paper_2208_01839_amd as sk
    c = si.config_nested_square(n_base=8, n_ref=2, n_sub=16, overlap=2)
    d = sk.analyze_schwarz(c.xy, c.tri, c.part, c.n_sub, 2, tile=tile, maps=True)
    G = node_graph(len(c.xy), c.tri)
    l2g, off, tiles, band = d["l2g"], 0, 0, 0
    for s in range(c.n_sub):
        nodes = subdomain_nodes(G, c.part, s, 2)
        seg = l2g[off:off + NC * len(nodes)]
        off += NC * len(nodes)
        order = seg[::NC] // NC
        assert sorted(order.tolist()) == nodes.tolist()          # the maps are the node set
        assert np.array_equal(seg, (NC * np.repeat(order, NC) + np.tile(np.arange(NC), len(order))))
        lo, hi = envelope(G, order, tile)
        assert np.all(np.diff(lo) >= 0) and np.all(lo <= np.arange(len(lo)))
        tiles += int(np.sum(hi - lo + 1))
        bw = int(np.max(hi - np.arange(len(hi))))
        band += len(lo) * (2 * bw + 1)
    assert off == len(l2g)
    assert d["factor_entries"] == tiles * tile * tile
    assert tiles <= band


def test_lu_fill_stays_inside_the_envelope():
    """Dense LU without pivoting of a diagonally dominant matrix with the
    subdomain's 5x5 block pattern: every nonzero of L and U lies in a
    stored tile."""
    import paper_2208_01839_amd as sk
    tile = 16
    c = si.config_nested_square(n_base=8, n_ref=1, n_sub=4, overlap=1)
    d = sk.analyze_schwarz(c.xy, c.tri, c.part, c.n_sub, 1, tile=tile, maps=True)
    G = node_graph(len(c.xy), c.tri)
    nodes = subdomain_nodes(G, c.part, 0, 1)
    order = d["l2g"][:NC * len(nodes)][::NC] // NC
    lo, hi = envelope(G, order, tile)
    B = (G[order][:, order] + sparse.identity(len(order))).toarray() != 0
    P = np.kron(B, np.ones((NC, NC), dtype=bool))
    rng = np.random.default_rng(1)
    n = P.shape[0]
    A = np.where(P, rng.uniform(-1.0, 1.0, P.shape), 0.0)
    A += np.diag(np.abs(A).sum(axis=1) + 1.0)
    for k in range(n - 1):  # LU in place (L strictly below, U on and above the diagonal)
        A[k + 1:, k] /= A[k, k]
        A[k + 1:, k + 1:] -= np.outer(A[k + 1:, k], A[k, k + 1:])
    I, J = np.nonzero(A)
    K, Jt = I // tile, J // tile
    assert np.all(Jt >= lo[K]) and np.all(Jt <= hi[K])
    # the envelope is strictly smaller than the dense lower/upper profile
    assert np.sum(hi - lo + 1) < len(lo) ** 2
