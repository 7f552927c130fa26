"""(k,h)-truss extraction, the plain way (TEST INFRASTRUCTURE ONLY, like the
rest of this package).

The (k,h)-truss is the set of edges whose h-trussness is at least k (Def. 4;
trusses are nested).  Its connected components are those of the graph formed
by exactly those edges; each component is named by its smallest vertex id.
The connectivity step is scipy's connected-components routine.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

NONE = 0xFFFFFFFF


def truss_components(g, t, k: int):
    """(label per edge, number of components) of the (k,h)-truss.

    g: graphgen.Graph (canonical edge order), t: trussness per edge.
    label[e] = smallest vertex of e's component if t[e] >= k, else 0xFFFFFFFF."""
    t = np.asarray(t, dtype=np.int64)
    if g.m == 0:
        return np.zeros(0, dtype=np.uint32), 0
    e = g.edges().astype(np.int64)           # (m, 2), canonical order
    keep = t >= k
    u, v = e[keep, 0], e[keep, 1]
    a = sp.coo_matrix((np.ones(u.size, dtype=np.int8), (u, v)), shape=(g.n, g.n)).tocsr()
    _, comp = connected_components(a, directed=False)
    # smallest vertex of every component
    smallest = np.full(comp.max() + 1 if g.n else 0, np.iinfo(np.int64).max, dtype=np.int64)
    np.minimum.at(smallest, comp, np.arange(g.n, dtype=np.int64))
    label = np.full(g.m, NONE, dtype=np.uint32)
    label[keep] = smallest[comp[u]].astype(np.uint32)
    touched = np.zeros(g.n, dtype=bool)
    touched[u] = True
    touched[v] = True
    count = int(np.unique(comp[touched]).size)
    return label, count
