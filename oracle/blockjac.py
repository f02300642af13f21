"""Block-Jacobi preconditioner (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Section "Preconditioning": a local block-Jacobi scheme whose blocks are
assembled from calls of the operator (Section "Memory and computation time
considerations": composing the preconditioner takes many N(q) calls).  Here
a block is a box of bx x by x bz grid cells with all nv variables, so it is
an nb x nb matrix, nb = nv*bx*by*bz, with local index
    l = var*(bx*by*bz) + (cz*by + cy)*bx + cx,
and blocks are numbered b = (kb*nby + jb)*nbx + ib.

For a shift s the block is
    B_b(s) = P_b J P_b^T + diag_add I + noise_std E_b - s I
on the block's interior DOFs, E_b a standard-normal matrix from the
counter-based generator (seeded, shared by all shifts), and the identity on
its wall DOFs (the operator is P J P: wall values are not unknowns, so no
noise, shift or diagonal term enters there and B_b(s)^{-1} restricted to the
interior is the inverse of the interior part).  The preconditioner applies
z = P blockdiag(B_b)^{-1} r.
"""
from __future__ import annotations

import numpy as np

from . import operator as opr
from . import philox


def block_layout(prob, bx, by, bz=1):
    nx, ny, nz = prob.n
    if prob.ndim == 2:
        bz = 1
    if nx % bx or ny % by or nz % bz:
        raise ValueError("grid not divisible by the block size")
    nbx, nby, nbz = nx // bx, ny // by, nz // bz
    cells = bx * by * bz
    nb = prob.nv * cells
    return dict(bx=bx, by=by, bz=bz, nbx=nbx, nby=nby, nbz=nbz,
                nblocks=nbx * nby * nbz, nb=nb, cells=cells)


def block_dof_index(prob, lay):
    """idx[b, l] = flat index of local DOF l of block b in the SoA vector."""
    nx, ny, nz = prob.n
    bx, by, bz = lay["bx"], lay["by"], lay["bz"]
    b = np.arange(lay["nblocks"])
    ib = b % lay["nbx"]
    jb = (b // lay["nbx"]) % lay["nby"]
    kb = b // (lay["nbx"] * lay["nby"])
    l = np.arange(lay["nb"])
    var = l // lay["cells"]
    cell = l % lay["cells"]
    cx = cell % bx
    cy = (cell // bx) % by
    cz = cell // (bx * by)
    i = ib[:, None] * bx + cx[None, :]
    j = jb[:, None] * by + cy[None, :]
    k = kb[:, None] * bz + cz[None, :]
    return ((var[None, :] * nz + k) * ny + j) * nx + i


def blocks_from_dense(prob, Jfull, lay):
    """B_b = P_b J P_b^T read from a dense n x n Jacobian (all DOFs)."""
    idx = block_dof_index(prob, lay)
    return Jfull[idx[:, :, None], idx[:, None, :]]


def probe_colours(prob, lay, reach=3):
    """Colours per axis so that two distinct blocks of one colour are more
    than `reach` cells apart along some axis: c_a = 1 + ceil(reach / w_a)."""
    cols = []
    widths = (lay["bx"], lay["by"], lay["bz"])
    counts = (lay["nbx"], lay["nby"], lay["nbz"])
    for a in range(3):
        if a >= prob.ndim or counts[a] == 1:
            cols.append(1)
            continue
        c = 1 + -(-reach // widths[a])
        if prob.bc[a] == opr.BC_PERIODIC and counts[a] % c:
            raise ValueError("periodic block count not divisible by the colour count")
        cols.append(min(c, counts[a]))
    return tuple(cols)


def blocks_by_probing(prob, jv, lay):
    """Extract all blocks with coloured probe vectors: for each colour and
    each local DOF l, one product J e where e has a 1 at DOF l of every
    block of that colour; the response on a block's rows is column l of its
    block.  jv(v) must return J v as an array of prob.shape."""
    cx, cy, cz = probe_colours(prob, lay)
    idx = block_dof_index(prob, lay)
    b = np.arange(lay["nblocks"])
    ib = b % lay["nbx"]
    jb = (b // lay["nbx"]) % lay["nby"]
    kb = b // (lay["nbx"] * lay["nby"])
    colour = ((kb % cz) * cy + (jb % cy)) * cx + (ib % cx)
    nb = lay["nb"]
    B = np.zeros((lay["nblocks"], nb, nb))
    for col in range(cx * cy * cz):
        sel = np.nonzero(colour == col)[0]
        if len(sel) == 0:
            continue
        for l in range(nb):
            e = np.zeros(prob.ndof)
            e[idx[sel, l]] = 1.0
            y = np.asarray(jv(e.reshape(prob.shape))).ravel()
            B[sel, :, l] = y[idx[sel]]
    return B


def block_wall_mask(prob, lay):
    """wall[b, l]: local DOF l of block b sits on a wall row.  Such DOFs are
    not unknowns of the operator P J P (their rows and columns of B_b are
    zero), so the shifted block keeps the identity there."""
    idx = block_dof_index(prob, lay)
    interior = np.tile(opr.interior_mask(prob).ravel(), prob.nv)
    return interior[idx] == 0.0


def shifted_blocks(B, shift, diag_add, noise_std, seed, stream=0, wall=None):
    """B_b(s) = B_b + diag_add I + noise_std E_b - s I on the block's interior
    DOFs, and the identity on its wall DOFs (wall = block_wall_mask(...); no
    noise, shift or diagonal term there), so that the block's inverse
    restricted to the interior is the inverse of its interior part."""
    nblocks, nb, _ = B.shape
    E = philox.block_noise(seed, nb, np.arange(nblocks), stream)
    out = B + noise_std * E + (diag_add - shift) * np.eye(nb)[None]
    if wall is not None:
        w = np.asarray(wall, dtype=bool)
        out = np.where(w[:, :, None] | w[:, None, :], 0.0, out)
        bi, li = np.nonzero(w)
        out[bi, li, li] = 1.0
    return out


def apply(prob, Bs, lay, r):
    """z = P blockdiag(Bs)^{-1} r (plain batched solve)."""
    idx = block_dof_index(prob, lay)
    rv = np.asarray(r, dtype=np.float64).ravel()
    zb = np.linalg.solve(Bs, rv[idx][..., None])[..., 0]
    z = np.zeros(prob.ndof)
    z[idx] = zb
    return opr.project(prob, z.reshape(prob.shape))
