"""Row orderings for BILU(0) and their level sets (section 2.2.2).

Parity: pinned by validity properties (tests): every colour class is an
independent set of the face graph, every face at level l > 0 has a lower
neighbour at level l - 1, and the colouring of a structured mesh uses six
colours (the minimum, since an element's six faces are pairwise coupled).

The paper reorders BILU(0) with minimum discarded fill (oracle/mdf.py, which
needs the values of K); BILU(0) takes the ordering as an explicit input, and
this module provides the two orders that depend on the pattern alone: the
natural face order and a greedy colouring order.  The greedy colouring visits faces in ascending id
and gives each the smallest colour not held by an already-coloured face that
shares an element with it; the order lists faces by (colour, face id).
"""
import numpy as np


def natural_order(tmesh):
    return np.arange(tmesh.n_face, dtype=np.int64)


def greedy_colours(tmesh):
    colour = -np.ones(tmesh.n_face, dtype=np.int64)
    for f in range(tmesh.n_face):
        used = {int(colour[g]) for g in tmesh.pattern[f] if g != f and colour[g] >= 0}
        c = 0
        while c in used:
            c += 1
        colour[f] = c
    return colour


def greedy_colour_order(tmesh):
    colour = greedy_colours(tmesh)
    return np.lexsort((np.arange(tmesh.n_face), colour)).astype(np.int64)


def level_sets(tmesh, order):
    """Level of each face in the lower-triangular dependency graph of ``order``."""
    pos = np.empty(tmesh.n_face, dtype=np.int64)
    pos[np.asarray(order)] = np.arange(tmesh.n_face)
    level = np.zeros(tmesh.n_face, dtype=np.int64)
    for f in order:
        lower = [level[g] for g in tmesh.pattern[f] if pos[g] < pos[f]]
        level[f] = 1 + max(lower) if lower else 0
    return level
