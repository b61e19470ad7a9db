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

    def __repr__(self):
        return f"StructuredHexMesh({self.nx}x{self.ny}x{self.nz})"
