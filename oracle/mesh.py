"""Trace-space bookkeeping for the oracle (parity pinned by closed-form counts).

The trace unknowns are grouped in units of b dofs (unit u holds dofs
u * b + l), and every element lists the units of its S local trace slots:
its t = S b trace dofs are those units' dofs in slot order.  The global
trace matrix K has a b x b block (u, w) exactly when units u and w appear
in a common element.  Two numberings are used (section 2.1):

* face-private (the block structure of the Newton system, section 2.2.1):
  a unit is a face with b = 5 (p+1)^2 dofs, S = 6 slots per element;
* IEDG: a unit is a trace node with b = m = 5 components, S = 6 (p+1)^2
  slots, nodes shared along interior faces (an element may list one node in
  several slots, where its own faces meet).
"""
import numpy as np


class TraceMesh:
    def __init__(self, elem_faces, n_face, b):
        self.elem_faces = np.asarray(elem_faces, dtype=np.int64)
        self.n_elem = self.elem_faces.shape[0]
        self.slots = self.elem_faces.shape[1]
        self.n_face = int(n_face)
        self.b = int(b)
        self.t = self.slots * self.b
        self.n_trace = self.n_face * self.b
        # elements touching each face, ascending element id
        self.face_elems = [[] for _ in range(self.n_face)]
        for e in range(self.n_elem):
            for a in range(self.slots):
                self.face_elems[self.elem_faces[e, a]].append((e, a))
        # block pattern: face -> sorted list of coupled faces (incl. itself)
        cols = [set() for _ in range(self.n_face)]
        for e in range(self.n_elem):
            fs = self.elem_faces[e]
            for f in fs:
                cols[f].update(int(g) for g in fs)
        self.pattern = [sorted(c) for c in cols]

    def element_dofs(self, e):
        """Global trace dof indices of element e (length t), local slot order
        (an index repeats where the element lists a unit in several slots)."""
        fs = self.elem_faces[e]
        return (fs[:, None] * self.b + np.arange(self.b)[None, :]).ravel()

    def nnzb(self):
        return sum(len(c) for c in self.pattern)
