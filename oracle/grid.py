"""Multi-level dense feature grid: trilinear interpolation (oracle side).

Sec. 3.1 (Eq. SDF_MLP): the geometry feature of a point is the concatenation
of the trilinearly interpolated features of every level, coarse to fine.
Supplementary "Second-order Grid Sampler": inside the voxel that contains the
point, with local coordinates (x, y, z) in [0, 1]^3 and the eight vertex
features stacked in bit order theta_{xyz} = [000, 001, 010, 011, 100, 101,
110, 111], the interpolated value is theta^T w(x) (Eq. trilinear_interp) with
the coefficient vector of Eq. coefficient_vector.  This module writes out that
coefficient vector, its Jacobian (Eq. coeff_jacobian, columns J1..J3) and the
off-diagonal Hessian entries h12, h13, h23 exactly as the supplementary states
them, so the tests can compare them with independent derivatives.

Conventions (readings where the paper is silent):
* levels share the box [p0, p1]; level l has voxel edge v_l and vertex counts
  (nx, ny, nz); vertex (i, j, k) sits at p0 + v_l (i, j, k) and is row
  (k ny + j) nx + i of that level's feature table;
* u = (x - p0) / v_l, cell origin i0 = clamp(floor(u), 0, n - 2), local
  coordinate f = u - i0 (so f = 1 on the box's upper faces);
* world-space derivatives carry the 1 / v_l factor of the change of variables.
"""
import torch

# corner c = 4 bx + 2 by + bz, the paper's theta_{xyz} bit order
CORNER_BITS = [((c >> 2) & 1, (c >> 1) & 1, c & 1) for c in range(8)]


def coefficient_vector(f):
    """w(x) in R^8 for local coordinates f [..., 3] (Eq. coefficient_vector)."""
    x, y, z = f[..., 0], f[..., 1], f[..., 2]
    return torch.stack([
        (1 - x) * (1 - y) * (1 - z),
        (1 - x) * (1 - y) * z,
        (1 - x) * y * (1 - z),
        (1 - x) * y * z,
        x * (1 - y) * (1 - z),
        x * (1 - y) * z,
        x * y * (1 - z),
        x * y * z,
    ], -1)


def coefficient_jacobian(f):
    """dw/dx as [..., 8, 3] with columns J1, J2, J3 (Eq. coeff_jacobian)."""
    x, y, z = f[..., 0], f[..., 1], f[..., 2]
    J1 = torch.stack([-(1 - y) * (1 - z), -(1 - y) * z, -y * (1 - z), -y * z,
                      (1 - y) * (1 - z), (1 - y) * z, y * (1 - z), y * z], -1)
    J2 = torch.stack([-(1 - x) * (1 - z), -(1 - x) * z, (1 - x) * (1 - z), (1 - x) * z,
                      -x * (1 - z), -x * z, x * (1 - z), x * z], -1)
    # the third column as re-derived from the coefficient rows (the printed
    # column has a stray parenthesis in its third entry)
    J3 = torch.stack([-(1 - x) * (1 - y), (1 - x) * (1 - y), -(1 - x) * y, (1 - x) * y,
                      -x * (1 - y), x * (1 - y), -x * y, x * y], -1)
    return torch.stack([J1, J2, J3], -1)


def coefficient_hessian(f, theta):
    """d^2 f/dx^2 [..., 3, 3] of f = theta^T w for 1-D features theta [..., 8].

    The diagonal is zero; h12, h13, h23 follow the supplementary's closed forms.
    """
    x, y, z = f[..., 0], f[..., 1], f[..., 2]
    t = [theta[..., c] for c in range(8)]
    # index map: t[0]=000 t[1]=001 t[2]=010 t[3]=011 t[4]=100 t[5]=101 t[6]=110 t[7]=111
    h12 = (1 - z) * (t[0] + t[6] - t[2] - t[4]) + z * (t[1] + t[7] - t[3] - t[5])
    h13 = (1 - y) * (t[0] + t[5] - t[1] - t[4]) + y * (t[2] + t[7] - t[3] - t[6])
    h23 = (1 - x) * (t[0] + t[3] - t[1] - t[2]) + x * (t[4] + t[7] - t[5] - t[6])
    zero = torch.zeros_like(h12)
    return torch.stack([torch.stack([zero, h12, h13], -1),
                        torch.stack([h12, zero, h23], -1),
                        torch.stack([h13, h23, zero], -1)], -2)


def cell_and_local(x, p0, voxel, dims, x32=None):
    """Cell origin (long [..., 3], no gradient) and local coordinates f [..., 3].

    The cell is an integer decision: at a face between two cells the
    interpolated value is continuous but its derivative in x jumps, so both
    implementations must pick the same cell.  With x32 (the float32 positions
    the device works on) the decision is taken as float32 arithmetic takes it,
    u = (x32 - p0) / voxel rounded to float32; the local coordinates are then
    u - i0 in the arithmetic of x."""
    p0t = torch.as_tensor(p0, dtype=x.dtype)
    u = (x - p0t) / voxel
    n = torch.as_tensor(dims, dtype=torch.long)
    if x32 is None:
        fl = torch.floor(u.detach()).long()
    else:
        import numpy as np
        u32 = (np.asarray(x32, dtype=np.float32).reshape(tuple(u.shape)) - np.asarray(p0, dtype=np.float32)) \
            / np.float32(voxel)
        fl = torch.from_numpy(np.floor(u32.astype(np.float32)).astype(np.int64))
    i0 = torch.minimum(fl.clamp(min=0), n - 2)
    f = u - i0.to(x.dtype)
    return i0, f


def corner_rows(i0, dims):
    """Feature-table rows of the 8 corners [..., 8] in theta_{xyz} order."""
    nx, ny, _ = dims
    rows = []
    for bx, by, bz in CORNER_BITS:
        rows.append(((i0[..., 2] + bz) * ny + (i0[..., 1] + by)) * nx + (i0[..., 0] + bx))
    return torch.stack(rows, -1)


def interp_level(table, x, p0, voxel, dims, x32=None):
    """Trilinear interpolation of one level: table [V, F], x [P, 3] -> [P, F]
    (x32: float32 positions that decide the cell, see cell_and_local)."""
    i0, f = cell_and_local(x, p0, voxel, dims, x32)
    w = coefficient_vector(f)                       # [P, 8]
    rows = corner_rows(i0, dims)                    # [P, 8]
    theta = table[rows]                             # [P, 8, F]
    return (w[..., None] * theta).sum(-2)


def interp_all(grid, layout, x, x32=None):
    """Concatenated features z = [V^0(x), ..., V^{L-1}(x)], coarsest level first."""
    out = []
    for l in range(layout.n_levels):
        nx, ny, nz = layout.dims[l]
        tab = grid[layout.offsets[l]:layout.offsets[l] + nx * ny * nz]
        out.append(interp_level(tab, x, layout.p0, layout.voxels[l], layout.dims[l], x32))
    return torch.cat(out, -1)


def interp_level_bruteforce(table, x, p0, voxel, dims):
    """Independent form: sum over *all* vertices of the tensor-product hat
    functions max(0, 1 - |u - i|); equals trilinear interpolation inside the box."""
    p0 = torch.as_tensor(p0, dtype=x.dtype)
    u = (x - p0) / voxel
    nx, ny, nz = dims
    hx = (1 - (u[:, 0, None] - torch.arange(nx, dtype=x.dtype)).abs()).clamp(min=0)
    hy = (1 - (u[:, 1, None] - torch.arange(ny, dtype=x.dtype)).abs()).clamp(min=0)
    hz = (1 - (u[:, 2, None] - torch.arange(nz, dtype=x.dtype)).abs()).clamp(min=0)
    w = hz[:, :, None, None] * hy[:, None, :, None] * hx[:, None, None, :]   # [P, nz, ny, nx]
    return w.reshape(x.shape[0], -1) @ table


def position_fp32(o32, t32, r32):
    """The point o + t r as the device forms it in float32 (product rounded,
    then sum rounded)."""
    import numpy as np
    o32 = np.asarray(o32, dtype=np.float32)
    r32 = np.asarray(r32, dtype=np.float32)
    t32 = np.asarray(t32, dtype=np.float32)
    return (o32 + (t32[..., None] * r32).astype(np.float32)).astype(np.float32)


def inside_box_fp32(o32, t32, r32, p0, p1):
    """Sample validity, decided in float32 as the device decides it: the point
    o + t r (product rounded, then sum rounded) must lie in the box."""
    import numpy as np
    o32 = np.asarray(o32, dtype=np.float32)
    r32 = np.asarray(r32, dtype=np.float32)
    t32 = np.asarray(t32, dtype=np.float32)
    x = (o32 + (t32[..., None] * r32).astype(np.float32)).astype(np.float32)
    lo = np.asarray(p0, dtype=np.float32)
    hi = np.asarray(p1, dtype=np.float32)
    return np.all((x >= lo) & (x <= hi), axis=-1)
