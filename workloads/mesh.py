"""Mesh generators: structured hexahedral boxes, Kuhn-split tetrahedral boxes,
the 16-node patch-test geometry, and boundary-face extraction.

This module holds topology and coordinates only.  It computes no shape
functions, volumes, areas or time steps: those belong to the method and are
computed independently by the oracle and by the GPU library.

Conventions
-----------
* Coordinates are float64 arrays ``x, y, z`` of length ``n_nodes`` (metres).
* Connectivity is int32, structure-of-arrays: ``conn[a, e]`` is the global
  node of local node ``a`` of element ``e`` (0-based).
* Hexahedron local order in natural coordinates (xi, eta, zeta):
  (---) (+--) (++-) (-+-) (--+) (+-+) (+++) (-++).
* Tetrahedra may have either orientation; consumers use |det|.
* Faces are int32 arrays ``faces[f, :]`` of 4 (quad) or 3 (triangle) nodes.
"""
from __future__ import annotations

import numpy as np

# Sign pattern of the hexahedron local nodes (xi, eta, zeta) in the order above.
HEX_SIGNS = np.array(
    [[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
     [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.int8)

# Local node lists of the six hexahedron faces (outward-ordered quads).
HEX_FACES = np.array(
    [[0, 3, 2, 1], [4, 5, 6, 7], [0, 1, 5, 4],
     [1, 2, 6, 5], [2, 3, 7, 6], [3, 0, 4, 7]], dtype=np.int64)

TET_FACES = np.array([[0, 2, 1], [0, 1, 3], [1, 2, 3], [0, 3, 2]], dtype=np.int64)


def grid_nodes(nx, ny, nz, lx, ly, lz):
    """Nodes of an (nx+1)x(ny+1)x(nz+1) lattice on [0,lx]x[0,ly]x[0,lz].

    Node id = i + (nx+1) * (j + (ny+1) * k).  Returns x, y, z (float64).
    """
    xs = np.linspace(0.0, lx, nx + 1)
    ys = np.linspace(0.0, ly, ny + 1)
    zs = np.linspace(0.0, lz, nz + 1)
    zz, yy, xx = np.meshgrid(zs, ys, xs, indexing="ij")
    return xx.ravel().copy(), yy.ravel().copy(), zz.ravel().copy()


def _nid(i, j, k, nx, ny):
    return i + (nx + 1) * (j + (ny + 1) * k)


def box_hex(nx, ny, nz, lx=1.0, ly=1.0, lz=1.0):
    """Structured box of nx*ny*nz 8-node hexahedra.

    Element id = i + nx * (j + ny * k).  Returns dict(x, y, z, conn[8, E]).
    """
    x, y, z = grid_nodes(nx, ny, nz, lx, ly, lz)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    conn = np.empty((8, i.size), dtype=np.int32)
    for a, (si, sj, sk) in enumerate(HEX_SIGNS):
        conn[a] = _nid(i + (si > 0), j + (sj > 0), k + (sk > 0), nx, ny)
    return dict(elem="hex8", x=x, y=y, z=z, conn=conn, shape=(nx, ny, nz))


# Kuhn (Freudenthal) split of the unit cube into 6 tetrahedra sharing the main
# diagonal (0,0,0)-(1,1,1): one tetrahedron per ordering of the three axis steps.
_KUHN_PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def box_tet_kuhn(nx, ny, nz, lx=1.0, ly=1.0, lz=1.0):
    """Structured box with every cell split into 6 Kuhn tetrahedra.

    The same split in every cell makes the mesh conforming.  Element id =
    6 * cell + p with p the axis-ordering index.  Returns dict(x, y, z, conn[4, E]).
    """
    x, y, z = grid_nodes(nx, ny, nz, lx, ly, lz)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    ncell = i.size
    conn = np.empty((4, 6 * ncell), dtype=np.int32)
    for p, perm in enumerate(_KUHN_PERMS):
        off = np.zeros((3, ncell), dtype=np.int64)
        cols = [_nid(i, j, k, nx, ny)]
        for axis in perm:
            off[axis] += 1
            cols.append(_nid(i + off[0], j + off[1], k + off[2], nx, ny))
        for a in range(4):
            conn[a, p::6] = cols[a]
    return dict(elem="tet4", x=x, y=y, z=z, conn=conn, shape=(nx, ny, nz))


def box_side_faces(mesh):
    """Boundary faces of a structured box mesh, with the box side of each face.

    Returns (faces[int32, F x nfn], side[int8, F]) where side is
    0:x=0 1:x=lx 2:y=0 3:y=ly 4:z=0 5:z=lz.  Quads for hex boxes; for Kuhn
    tetrahedra each boundary square is split along the diagonal that joins its
    low corner to its high corner, which is the diagonal the Kuhn cells use.
    """
    nx, ny, nz = mesh["shape"]
    faces, sides = [], []

    def quads(axis, level):
        # the two in-plane axes, in increasing order
        u, v = [a for a in range(3) if a != axis]
        n = [nx, ny, nz]
        vv, uu = np.meshgrid(np.arange(n[v]), np.arange(n[u]), indexing="ij")
        uu, vv = uu.ravel(), vv.ravel()

        def node(du, dv):
            idx = [None, None, None]
            idx[axis] = np.full(uu.size, level)
            idx[u] = uu + du
            idx[v] = vv + dv
            return _nid(idx[0], idx[1], idx[2], nx, ny)

        return node(0, 0), node(1, 0), node(1, 1), node(0, 1)

    for side in range(6):
        axis, hi = divmod(side, 2)
        level = [nx, ny, nz][axis] if hi else 0
        c00, c10, c11, c01 = quads(axis, level)
        if mesh["elem"] == "hex8":
            f = np.stack([c00, c10, c11, c01], axis=1)
        else:
            f = np.concatenate([np.stack([c00, c10, c11], axis=1),
                                np.stack([c00, c11, c01], axis=1)], axis=0)
        faces.append(f)
        sides.append(np.full(f.shape[0], side, dtype=np.int8))
    return np.concatenate(faces).astype(np.int32), np.concatenate(sides)


def boundary_faces(mesh):
    """Faces that belong to exactly one element (generic, any mesh).

    Returns faces[int32, F x nfn] with node tuples in element-local order.
    Used to cross-check :func:`box_side_faces` and for unstructured meshes.
    """
    table = HEX_FACES if mesh["elem"] == "hex8" else TET_FACES
    conn = mesh["conn"]
    allf = np.concatenate([conn[list(t)].T for t in table], axis=0)
    key = np.sort(allf, axis=1)
    _, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    once = cnt[inv.ravel()] == 1
    return allf[once].astype(np.int32)


def boundary_nodes(mesh):
    """Sorted ids of nodes that lie on a boundary face."""
    return np.unique(boundary_faces(mesh))


def jitter_interior(mesh, amp, seed):
    """Copy of a box mesh with every node off the boundary moved by a seeded
    uniform offset of up to amp times the local spacing in each direction (a
    distorted, still valid hexahedral or tetrahedral mesh for amp well below
    1/2)."""
    g = np.random.default_rng(seed)
    x, y, z = mesh["x"].copy(), mesh["y"].copy(), mesh["z"].copy()
    inner = np.ones(x.size, bool)
    inner[boundary_nodes(mesh)] = False
    for c in (x, y, z):
        h = np.diff(np.unique(np.round(c, 12))).min()
        c[inner] += amp * h * g.uniform(-1.0, 1.0, inner.sum())
    return dict(mesh, x=x, y=y, z=z)


# Patch-test geometry (Sec. 4.1, Fig. 2(c)): eight unit-cube corners and
# eight interior nodes, loaded from the text fixture that transcribes the
# printed coordinates.
def patch_nodes(path):
    """Read the 16 patch-test node coordinates (1-based ids in the file)."""
    rows = []
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(v) for v in line.split()])
    arr = np.array(rows)
    order = np.argsort(arr[:, 0])
    arr = arr[order]
    assert arr.shape == (16, 4)
    return arr[:, 1].copy(), arr[:, 2].copy(), arr[:, 3].copy()


def patch_hex(x, y, z):
    """Seven-hexahedron patch: the inner hexahedron (nodes 9-16) plus one
    hexahedron joining each cube face to the matching inner face.

    The figure with the connectivity is not available, so this is the
    construction chosen for the test; node ids are 0-based here.
    """
    outer = np.array([0, 1, 3, 2, 4, 5, 7, 6])      # corners in local hex order
    inner = np.arange(8, 16)                        # nodes 9..16 in local hex order
    elems = [inner]
    for f in HEX_FACES:
        # HEX_FACES quads are ordered with the normal pointing out of the cube;
        # reversed, the cube-face quad is counter-clockwise seen from the inner
        # hexahedron, so it is the bottom (zeta=-1) face of the joining element
        # and the matching inner quad, in the same corner order, is its top.
        o = outer[f[::-1]]
        i = inner[f[::-1]]
        elems.append(np.concatenate([o, i]))
    conn = np.array(elems, dtype=np.int32).T.copy()
    return dict(elem="hex8", x=x, y=y, z=z, conn=conn)


def patch_tet(x, y, z):
    """Tetrahedral patch: a Delaunay tetrahedralisation of the 16 nodes."""
    from scipy.spatial import Delaunay
    pts = np.stack([x, y, z], axis=1)
    tri = Delaunay(pts)
    conn = tri.simplices.T.astype(np.int32).copy()
    return dict(elem="tet4", x=x, y=y, z=z, conn=conn)


def concatenate(meshes, offsets=None):
    """Concatenate disjoint meshes into one (node ids shifted per instance).

    ``offsets`` optionally translates each instance so the instances do not
    overlap in space.  Returns the merged mesh plus per-node and per-element
    instance ids and the node/element start of every instance.
    """
    elem = meshes[0]["elem"]
    xs, ys, zs, conns, ni, ei = [], [], [], [], [], []
    node_start, elem_start = [0], [0]
    base = 0
    for m, mesh in enumerate(meshes):
        assert mesh["elem"] == elem
        dx, dy, dz = (0.0, 0.0, 0.0) if offsets is None else offsets[m]
        xs.append(mesh["x"] + dx)
        ys.append(mesh["y"] + dy)
        zs.append(mesh["z"] + dz)
        conns.append(mesh["conn"].astype(np.int64) + base)
        n = mesh["x"].size
        e = mesh["conn"].shape[1]
        ni.append(np.full(n, m, dtype=np.int32))
        ei.append(np.full(e, m, dtype=np.int32))
        base += n
        node_start.append(base)
        elem_start.append(elem_start[-1] + e)
    return dict(elem=elem, x=np.concatenate(xs), y=np.concatenate(ys),
                z=np.concatenate(zs),
                conn=np.concatenate(conns, axis=1).astype(np.int32),
                node_instance=np.concatenate(ni), elem_instance=np.concatenate(ei),
                node_start=np.array(node_start, dtype=np.int64),
                elem_start=np.array(elem_start, dtype=np.int64))
