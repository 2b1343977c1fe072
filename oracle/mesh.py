"""Surface extraction from the SDF (oracle side; test infrastructure only).

The reconstructed surface is the zero level set of the SDF phi (Sec. 3.1);
the paper extracts it with marching cubes on a 1 cm lattice for evaluation.
This restates the extraction as marching tetrahedra, whose case analysis is
short enough to write out here:

* the SDF is sampled at the lattice points p0 + h (i, j, k), i < nx, j < ny,
  k < nz, stored [k][j][i] (x fastest);
* each cube (i, j, k) of 8 lattice points (corner c = bx + 2 by + 4 bz) is
  split into the six tetrahedra around its main diagonal 0-7:
  (0,1,3,7), (0,3,2,7), (0,2,6,7), (0,6,4,7), (0,4,5,7), (0,5,1,7); every
  cube splits each face along the diagonal through the face's lowest and
  highest corners, so neighbouring cubes agree on shared faces;
* a corner is inside when phi < 0; a tetrahedron with one corner on one side
  and three on the other yields one triangle through the three edges that
  cross, one with two and two yields the quadrilateral through its four
  crossing edges as two triangles (edges in cyclic order a0b0, a0b1, a1b1,
  a1b0 for inside corners a0, a1 and outside corners b0, b1);
* an edge (p, q) crosses at p + phi_p / (phi_p - phi_q) (q - p), the zero of
  the linear interpolation along it.

Triangles are returned as [T, 3, 3] float64 vertex positions, in no
particular order (orientation is not fixed).
"""
import numpy as np
import torch

TETS = np.array([[0, 1, 3, 7], [0, 3, 2, 7], [0, 2, 6, 7], [0, 6, 4, 7], [0, 4, 5, 7], [0, 5, 1, 7]])
CORNER = np.array([[c & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)])


def lattice_points(p0, h, dims):
    """[nz * ny * nx, 3] lattice positions, x fastest."""
    nx, ny, nz = dims
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    idx = np.stack([i, j, k], -1).reshape(-1, 3).astype(np.float64)
    return np.asarray(p0, dtype=np.float64) + h * idx


def field_sdf(grid, mlp, layout):
    """phi(x) of the grid and decoders (float64), for points x [P, 3]."""
    from . import decoder as D, grid as G
    P = D.unpack(torch.as_tensor(mlp, dtype=torch.float64))
    g = torch.as_tensor(grid, dtype=torch.float64)

    def f(x):
        z = G.interp_all(g, layout, torch.as_tensor(np.asarray(x, dtype=np.float64)))
        return D.geometry(z, P)[:, 0].numpy()
    return f


def _cross(pa, pb, fa, fb):
    return pa + (fa / (fa - fb))[:, None] * (pb - pa)


def marching_tetrahedra(phi, p0, h):
    """phi: [nz, ny, nx] lattice values -> triangles [T, 3, 3]."""
    phi = np.asarray(phi, dtype=np.float64)
    nz, ny, nx = phi.shape
    k, j, i = np.meshgrid(np.arange(nz - 1), np.arange(ny - 1), np.arange(nx - 1), indexing="ij")
    base = np.stack([i.ravel(), j.ravel(), k.ravel()], -1)                         # [C, 3]
    corner_idx = base[:, None, :] + CORNER[None, :, :]                             # [C, 8, 3]
    vals = phi[corner_idx[..., 2], corner_idx[..., 1], corner_idx[..., 0]]        # [C, 8]
    pos = np.asarray(p0, dtype=np.float64) + h * corner_idx.astype(np.float64)     # [C, 8, 3]
    tris = []
    for tet in TETS:
        v = vals[:, tet]                                                           # [C, 4]
        p = pos[:, tet]                                                            # [C, 4, 3]
        inside = v < 0
        n_in = inside.sum(1)
        for cnt in (1, 3):
            sel = np.nonzero(n_in == cnt)[0]
            if sel.size == 0:
                continue
            lone_mask = inside[sel] if cnt == 1 else ~inside[sel]
            lone = np.argmax(lone_mask, 1)                                         # the corner alone on its side
            others = np.array([[q for q in range(4) if q != a] for a in range(4)])[lone]
            pl = p[sel, lone]
            fl = v[sel, lone]
            tri = np.stack([_cross(pl, p[sel, others[:, e]], fl, v[sel, others[:, e]]) for e in range(3)], 1)
            tris.append(tri)
        sel = np.nonzero(n_in == 2)[0]
        if sel.size:
            ins = inside[sel]
            order = np.argsort(~ins, axis=1, kind="stable")                        # inside corners first
            a0, a1, b0, b1 = (order[:, q] for q in range(4))
            r = np.arange(sel.size)

            def X(a, b):
                return _cross(p[sel, a], p[sel, b], v[sel, a], v[sel, b])
            e00, e01, e11, e10 = X(a0, b0), X(a0, b1), X(a1, b1), X(a1, b0)
            del r
            tris.append(np.stack([e00, e01, e11], 1))
            tris.append(np.stack([e00, e11, e10], 1))
    if not tris:
        return np.zeros((0, 3, 3))
    return np.concatenate(tris, 0)
