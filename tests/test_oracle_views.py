"""Pins of the per-PE view (Sec. 4.1 directed: a PE's row chunk; Sec. 4.2
undirected: the chunk row and column of its section): against the whole
graph, view r is exactly the set of edges with an endpoint in section r; the
views cover the graph, each undirected edge between two sections twice and
every other edge once; and the view's chunk counts come from the chunks' own
root paths (no communication)."""
import numpy as np
import pytest


def section_of(v, n, P):
    # section r holds vertices [floor(r n / P), floor((r + 1) n / P))
    bounds = np.array([(i * n) // P for i in range(P + 1)], dtype=np.int64)
    return np.searchsorted(bounds, v.astype(np.int64), side="right") - 1


CASES = [(60, 0, 500, 0.0, True, 5), (60, 0, 700, 0.0, False, 5), (97, 1, 0, 0.05, False, 7),
         (40, 1, 0, 0.2, True, 4), (33, 0, 200, 0.0, False, 1), (128, 0, 4000, 0.0, False, 16)]


@pytest.mark.parametrize("n,model,m,p,directed,P", CASES)
def test_views_are_the_incident_edges(kgref, n, model, m, p, directed, P):
    I = kgref.inst(n, m=m, p=p, directed=directed, seed=3, chunks=P, model=model)
    E = kgref.generate(I)
    su, sv = section_of(E[:, 0], n, P), section_of(E[:, 1], n, P)
    total = 0
    for r in range(P):
        V = kgref.pe_view(I, r)
        total += len(V)
        want = E[(su == r) | (sv == r)] if not directed else E[su == r]
        # the view's chunks are exactly those holding these edges, in
        # canonical order: the sequences agree, not only the sets
        assert np.array_equal(V, want), r
    cross = int(np.sum(su != sv)) if not directed else 0
    assert total == len(E) + cross


def test_view_counts_are_root_paths(kgref):
    I = kgref.inst(500, m=20000, directed=False, seed=9, chunks=12)
    counts = kgref.chunk_counts(I)            # the whole tree, expanded once
    for r in (0, 5, 11):
        for c in kgref.view_chunks(I, r):
            assert kgref.chunk_count_path(I, c) == counts[c]


def test_view_chunks_cover_row_and_column(kgref):
    P = 6
    I = kgref.inst(50, m=100, directed=False, seed=1, chunks=P)
    cells = {}
    o = 0
    for i in range(P):
        for j in range(i, P):
            cells[o] = (i, j)
            o += 1
    for r in range(P):
        got = [cells[c] for c in kgref.view_chunks(I, r)]
        assert got == [(i, r) for i in range(r)] + [(r, j) for j in range(r, P)]
