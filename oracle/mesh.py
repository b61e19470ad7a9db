"""Trace-space bookkeeping for the oracle (parity pinned by closed-form counts).

The trace unknowns live on faces.  Following the block structure of the
Newton system (section 2.2.1), each face carries b = 5 (p+1)^2 private trace
dofs, numbered f * b + l, and an element's t = 6 b trace dofs are its six
faces' dofs in local face order.  The global trace matrix K therefore has a
b x b block (f, g) exactly when faces f and g belong to a common element.
"""
import numpy as np


class TraceMesh:
    def __init__(self, elem_faces, n_face, b):
        self.elem_faces = np.asarray(elem_faces, dtype=np.int64)
        self.n_elem = self.elem_faces.shape[0]
        self.n_face = int(n_face)
        self.b = int(b)
        self.t = 6 * self.b
        self.n_trace = self.n_face * self.b
        # elements touching each face, ascending element id
        self.face_elems = [[] for _ in range(self.n_face)]
        for e in range(self.n_elem):
            for a in range(6):
                self.face_elems[self.elem_faces[e, a]].append((e, a))
        # block pattern: face -> sorted list of coupled faces (incl. itself)
        cols = [set() for _ in range(self.n_face)]
        for e in range(self.n_elem):
            fs = self.elem_faces[e]
            for f in fs:
                cols[f].update(int(g) for g in fs)
        self.pattern = [sorted(c) for c in cols]

    def element_dofs(self, e):
        """Global trace dof indices of element e (length t), local face order."""
        fs = self.elem_faces[e]
        return (fs[:, None] * self.b + np.arange(self.b)[None, :]).ravel()

    def nnzb(self):
        return sum(len(c) for c in self.pattern)
