"""Structured hexahedral mesh topology (element -> face incidence).

Numbering used throughout the repository:
* element (i, j, k), 0 <= i < nx, 0 <= j < ny, 0 <= k < nz, has id
  (i * ny + j) * nz + k;
* faces are numbered direction-major.  x-faces (i in [0, nx], j, k) take ids
  (i * ny + j) * nz + k; y-faces (i, j in [0, ny], k) follow at offset
  Nx = (nx + 1) * ny * nz with local id (i * (ny + 1) + j) * nz + k; z-faces
  (i, j, k in [0, nz]) follow at offset Nx + Ny, Ny = nx * (ny + 1) * nz, with
  local id (i * ny + j) * (nz + 1) + k;
* an element lists its faces in the local order (-x, +x, -y, +y, -z, +z).

The mesh is not periodic: faces on the outer boundary touch one element.
"""
import numpy as np


class StructuredHexMesh:
    def __init__(self, nx, ny, nz):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.n_elem = self.nx * self.ny * self.nz
        self.n_xface = (self.nx + 1) * self.ny * self.nz
        self.n_yface = self.nx * (self.ny + 1) * self.nz
        self.n_zface = self.nx * self.ny * (self.nz + 1)
        self.n_face = self.n_xface + self.n_yface + self.n_zface

    def xface(self, i, j, k):
        return (i * self.ny + j) * self.nz + k

    def yface(self, i, j, k):
        return self.n_xface + (i * (self.ny + 1) + j) * self.nz + k

    def zface(self, i, j, k):
        return self.n_xface + self.n_yface + (i * self.ny + j) * (self.nz + 1) + k

    def elem_faces(self):
        """int32 array [n_elem, 6] of face ids in local order (-x,+x,-y,+y,-z,+z)."""
        i, j, k = np.meshgrid(np.arange(self.nx), np.arange(self.ny),
                              np.arange(self.nz), indexing="ij")
        i, j, k = i.ravel(), j.ravel(), k.ravel()
        ef = np.stack([self.xface(i, j, k), self.xface(i + 1, j, k),
                       self.yface(i, j, k), self.yface(i, j + 1, k),
                       self.zface(i, j, k), self.zface(i, j, k + 1)], axis=1)
        return np.ascontiguousarray(ef.astype(np.int32))

    def face_geometry(self):
        """Per face: (direction 0/1/2, index along the face normal)."""
        d = np.empty(self.n_face, dtype=np.int32)
        idx = np.empty(self.n_face, dtype=np.int32)
        i, j, k = np.meshgrid(np.arange(self.nx + 1), np.arange(self.ny),
                              np.arange(self.nz), indexing="ij")
        f = self.xface(i, j, k).ravel()
        d[f], idx[f] = 0, i.ravel()
        i, j, k = np.meshgrid(np.arange(self.nx), np.arange(self.ny + 1),
                              np.arange(self.nz), indexing="ij")
        f = self.yface(i, j, k).ravel()
        d[f], idx[f] = 1, j.ravel()
        i, j, k = np.meshgrid(np.arange(self.nx), np.arange(self.ny),
                              np.arange(self.nz + 1), indexing="ij")
        f = self.zface(i, j, k).ravel()
        d[f], idx[f] = 2, k.ravel()
        return d, idx

    def face_slabs(self, n_sub):
        """Partition of the faces into n_sub subdomains (input data for the
        restricted additive Schwarz preconditioner, in place of a graph
        partitioner): elements go to n_sub slabs of equal width along x
        (slab of element (i, j, k) = i * n_sub // nx), and a face to the slab
        of the lowest-numbered element it bounds.  Returns int32 [n_face]."""
        if not 1 <= n_sub <= self.nx:
            raise ValueError(f"n_sub must be in [1, {self.nx}]")
        ef = self.elem_faces()
        slab_of_elem = (np.arange(self.n_elem) // (self.ny * self.nz)) * n_sub // self.nx
        part = np.full(self.n_face, -1, dtype=np.int32)
        for e in range(self.n_elem):          # ascending: the first element wins
            for f in ef[e]:
                if part[f] < 0:
                    part[f] = slab_of_elem[e]
        return part

    def iedg_trace_nodes(self, p, m=5):
        """Trace numbering of the IEDG method (section 2.1: the trace space is
        continuous on interior faces and discontinuous on boundary faces),
        with m components per node.  Returns (elem_nodes int32 [E][6 (p+1)^2],
        n_nodes): the global node of every local trace slot; local trace dof
        slot * m + c holds component c of that node, so an element's t =
        6 (p+1)^2 m trace dofs keep the face-private layout (face a, then node
        q = u (p+1) + v of its (p+1) x (p+1) grid, u and v along the face's
        two tangential axes in increasing order of x, y, z).
        A node of an interior face is a point of the (p nx + 1) x (p ny + 1) x
        (p nz + 1) lattice and is shared by every interior face through it
        (so also by the faces of one element that meet at an edge); a
        boundary face has (p+1)^2 nodes of its own.  Nodes are numbered in
        order of first appearance over faces in id order."""
        p1 = p + 1
        d, idx = self.face_geometry()
        ef = self.elem_faces()
        # face -> lower corner (element coordinates) and tangential axes
        corner = np.zeros((self.n_face, 3), dtype=np.int64)
        for e in range(self.n_elem):
            ei, ej, ek = e // (self.ny * self.nz), (e // self.nz) % self.ny, e % self.nz
            for a in range(6):
                f = ef[e, a]
                c = [ei, ej, ek]
                c[d[f]] = idx[f]
                corner[f] = c
        nmax = (self.nx, self.ny, self.nz)
        boundary = np.array([idx[f] == 0 or idx[f] == nmax[d[f]] for f in range(self.n_face)])
        face_nodes = np.empty((self.n_face, p1 * p1), dtype=np.int64)
        lattice = {}
        count = 0
        for f in range(self.n_face):
            tang = [x for x in range(3) if x != d[f]]
            for u in range(p1):
                for v in range(p1):
                    if boundary[f]:
                        face_nodes[f, u * p1 + v] = count
                        count += 1
                        continue
                    P = [p * corner[f, x] for x in range(3)]
                    P[tang[0]] += u
                    P[tang[1]] += v
                    key = tuple(P)
                    if key not in lattice:
                        lattice[key] = count
                        count += 1
                    face_nodes[f, u * p1 + v] = lattice[key]
        elem_nodes = face_nodes[ef].reshape(self.n_elem, 6 * p1 * p1)
        return np.ascontiguousarray(elem_nodes.astype(np.int32)), count

    def __repr__(self):
        return f"StructuredHexMesh({self.nx}x{self.ny}x{self.nz})"
