"""Oracle: assembly of the H-field nodal finite element system (CPU, FP64).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
module; only the test suite, the smoke check and the benchmark's CPU-baseline
leg do.  It shares no code with the HIP library.

What is computed (paper section 2, eqs. (1)-(4)), with the readings used:

* Unknown: the total magnetic field H, three complex components per mesh
  node, on first-order (8-node trilinear) hexahedra (section 1).
* Volume operator, standard curl sign (eq. (4) multiplied by -1, which makes
  eq. (4)'s "+k0^2 mass" consistent with eq. (1)'s "-k0^2 mass"):
      a(W, H) = int (1/eps_r) curl W . curl H  +  s int div W div H
                - k0^2 int mu_r W . H
  with vector test functions W = N_a e_i.  The grad-div penalty of eq. (2)
  enters with weight s (the paper gives none; default 1).  The penalty's
  surface integral is dropped: its natural condition div H = 0 holds for the
  true field when mu_r = 1, and the matrix stays complex-symmetric.
* Outer faces tagged ABC (eq. (3), second-order Engquist-Majda):
      int W . g(H) dS,  g(H) = j k0 H_t - (j / 2k0) lap_t H_t,
  the surface Laplacian integrated by parts on each face (edge terms
  dropped), i.e. j k0 int W_t . H_t + (j / 2k0) int grad_t W_t : grad_t H_t.
* Total-field right-hand side (eq. (4), sign read so that an empty box is
  solved by the incident field):
      int_{S_ext} W . [ g(H_i) - n x curl H_i ] dS.
* PEC elements are removed; PEC is a natural condition for H, so S_pec
  carries no term.  Faces not tagged ABC carry no term either.
* Symmetry planes (section 3.1.3): an outer face tagged 2 is a symmetry
  plane, n . H = 0 (eq. (6a)); one tagged 3 an antisymmetry plane,
  n x H = 0 (eq. (6b)).  These are essential conditions: on every active
  node of such a face the constrained components (the normal one, or the
  two tangential ones) are fixed to zero by the usual elimination, their
  rows and columns replaced by those of the identity and their right-hand
  side entries by zero, which keeps the matrix complex-symmetric.  The
  remaining components keep their natural conditions.
* Quadrature: 2x2x2 Gauss points in volumes, 2x2 on faces; the incident
  field is evaluated exactly at the face Gauss points.

Indexing: element (ex, ey, ez) of an nx*ny*nz box; node (i, j, k) at
origin + (i hx, j hy, k hz).  Arrays of elements are shaped (nz, ny, nx)
(x fastest).  Active nodes (incident to a non-PEC element) are numbered in
lexicographic grid order with x fastest; unknown = 3 * node + component.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

# Local node a of an element sits at offset (ax, ay, az); a = ax + 2 ay + 4 az.
LOCAL_NODES = np.array([(ax, ay, az) for az in (0, 1) for ay in (0, 1) for ax in (0, 1)], dtype=np.int64)

_G = 1.0 / math.sqrt(3.0)
GAUSS_POINTS_UNIT = np.array([0.5 * (1.0 - _G), 0.5 * (1.0 + _G)])  # on [0, 1]
GAUSS_WEIGHTS_UNIT = np.array([0.5, 0.5])


def _hat(t, which):
    """1-D linear Lagrange function on [0, 1]: 1 - t (which = 0) or t (which = 1),
    and its derivative."""
    if which == 0:
        return 1.0 - t, -1.0
    return t, 1.0


def volume_basis_at(xi, h):
    """Values (8,) and physical gradients (8, 3) of the trilinear shape
    functions at a point xi of the unit reference cube, element size h."""
    N = np.empty(8)
    dN = np.empty((8, 3))
    for a, (ax, ay, az) in enumerate(LOCAL_NODES):
        fx, gx = _hat(xi[0], ax)
        fy, gy = _hat(xi[1], ay)
        fz, gz = _hat(xi[2], az)
        N[a] = fx * fy * fz
        dN[a] = (gx * fy * fz / h[0], fx * gy * fz / h[1], fx * fy * gz / h[2])
    return N, dN


def element_matrices(h):
    """24 x 24 element matrices of a box element of size h = (hx, hy, hz),
    row/column index 3 a + i for the vector basis function N_a e_i:

      Kc = int curl(N_a e_i) . curl(N_b e_j)     (curl-curl)
      Kd = int div(N_a e_i) div(N_b e_j)          (grad-div penalty)
      Km = int (N_a e_i) . (N_b e_j)              (mass)

    by 2x2x2 Gauss quadrature, literally from curl(N e_i) = grad N x e_i and
    div(N e_i) = dN/dx_i."""
    h = np.asarray(h, dtype=np.float64)
    detJ = h[0] * h[1] * h[2]
    E = np.eye(3)
    Kc = np.zeros((24, 24))
    Kd = np.zeros((24, 24))
    Km = np.zeros((24, 24))
    for wx, px in zip(GAUSS_WEIGHTS_UNIT, GAUSS_POINTS_UNIT):
        for wy, py in zip(GAUSS_WEIGHTS_UNIT, GAUSS_POINTS_UNIT):
            for wz, pz in zip(GAUSS_WEIGHTS_UNIT, GAUSS_POINTS_UNIT):
                w = wx * wy * wz * detJ
                N, dN = volume_basis_at((px, py, pz), h)
                curl = np.zeros((24, 3))
                div = np.zeros(24)
                val = np.zeros((24, 3))
                for a in range(8):
                    for i in range(3):
                        curl[3 * a + i] = np.cross(dN[a], E[i])
                        div[3 * a + i] = dN[a, i]
                        val[3 * a + i] = N[a] * E[i]
                Kc += w * curl @ curl.T
                Kd += w * np.outer(div, div)
                Km += w * val @ val.T
    return Kc, Kd, Km


# Outer faces: index f -> (normal axis, side); side 0 = minimum coordinate.
FACES = [(0, 0), (0, 1), (1, 0), (1, 1), (2, 0), (2, 1)]

# Outer-face tags: 0 ABC (eq. (3)), 1 natural (no term), 2 symmetry plane
# n . H = 0 (eq. (6a)), 3 antisymmetry plane n x H = 0 (eq. (6b)).
FACE_TAG_ABC, FACE_TAG_NATURAL, FACE_TAG_SYM, FACE_TAG_ANTISYM = 0, 1, 2, 3


def constrained_unknowns(prob):
    """Boolean mask (n_unknowns,) of the unknowns the symmetry planes fix to
    zero (section 3.1.3): on every active node of a face tagged 2 the
    component along the face normal (n . H = 0, eq. (6a)); on a face tagged
    3 the two tangential components (n x H = 0, eq. (6b)).  A node on two
    such faces collects both sets."""
    mesh = Mesh(prob)
    k, j, i = np.nonzero(mesh.node_active)
    ijk = (i, j, k)
    mask = np.zeros((mesh.n_nodes, 3), dtype=bool)
    for f in range(6):
        tag = prob.faces[f]
        if tag not in (FACE_TAG_SYM, FACE_TAG_ANTISYM):
            continue
        axis, side = FACES[f]
        n_axis = (mesh.nx, mesh.ny, mesh.nz)[axis]
        on = ijk[axis] == (0 if side == 0 else n_axis)
        comps = [axis] if tag == FACE_TAG_SYM else [c for c in range(3) if c != axis]
        for c in comps:
            mask[on, c] = True
    return mask.ravel()


def apply_constraints(A, constrained):
    """Elimination of unknowns fixed to zero: their rows and columns become
    those of the identity (P A P + I_c with P the projector on the free
    unknowns)."""
    if not constrained.any():
        return A
    free = sp.diags((~constrained).astype(np.float64))
    fixed = sp.diags(constrained.astype(np.float64))
    return (free @ A @ free + fixed).tocsr()


def face_local_nodes(axis, side):
    """Local element nodes lying on the element face normal to `axis` at `side`."""
    return np.array([a for a in range(8) if LOCAL_NODES[a, axis] == side], dtype=np.int64)


def face_basis_at(eta, axis, side, h):
    """Values (4,) and tangential gradients (4, 3) (normal component 0) of the
    element's shape functions restricted to one face, at reference face point
    eta (two coordinates in [0, 1], along the two tangential axes in
    increasing order)."""
    tang = [t for t in range(3) if t != axis]
    xi = np.zeros(3)
    xi[axis] = float(side)
    xi[tang[0]], xi[tang[1]] = eta
    N, dN = volume_basis_at(xi, h)
    nodes = face_local_nodes(axis, side)
    g = dN[nodes].copy()
    g[:, axis] = 0.0
    return N[nodes], g


def face_matrices(axis, h):
    """4 x 4 face mass Mf = int N_a N_b dS and tangential stiffness
    Sf = int grad_t N_a . grad_t N_b dS on a face normal to `axis`
    (2x2 Gauss; face-local order = face_local_nodes(axis, side))."""
    h = np.asarray(h, dtype=np.float64)
    tang = [t for t in range(3) if t != axis]
    area = h[tang[0]] * h[tang[1]]
    Mf = np.zeros((4, 4))
    Sf = np.zeros((4, 4))
    for w1, p1 in zip(GAUSS_WEIGHTS_UNIT, GAUSS_POINTS_UNIT):
        for w2, p2 in zip(GAUSS_WEIGHTS_UNIT, GAUSS_POINTS_UNIT):
            w = w1 * w2 * area
            N, g = face_basis_at((p1, p2), axis, 0, h)
            Mf += w * np.outer(N, N)
            Sf += w * g @ g.T
    return Mf, Sf


class Mesh:
    """Active-element / active-node bookkeeping of a problem (see module doc)."""

    def __init__(self, prob):
        self.prob = prob
        self.nx, self.ny, self.nz = prob.nx, prob.ny, prob.nz
        self.h = np.asarray(prob.h, dtype=np.float64)
        self.origin = np.asarray(prob.origin, dtype=np.float64)
        pec = np.asarray(prob.pec).reshape(self.nz, self.ny, self.nx)
        self.active_elem = pec == 0
        node_active = np.zeros((self.nz + 1, self.ny + 1, self.nx + 1), dtype=bool)
        for ax, ay, az in LOCAL_NODES:
            node_active[az:az + self.nz, ay:ay + self.ny, ax:ax + self.nx] |= self.active_elem
        self.node_active = node_active
        self.node_id = np.full(node_active.shape, -1, dtype=np.int64)
        self.n_nodes = int(node_active.sum())
        self.node_id[node_active] = np.arange(self.n_nodes)
        self.n_unknowns = 3 * self.n_nodes
        ez, ey, ex = np.nonzero(self.active_elem)
        self.elem_ijk = np.stack([ex, ey, ez], axis=1)          # (E, 3)
        # global node id of each local node of each active element
        self.elem_nodes = np.stack(
            [self.node_id[ez + az, ey + ay, ex + ax] for ax, ay, az in LOCAL_NODES], axis=1)

    def node_coords(self):
        """Physical coordinates (n_nodes, 3) of the active nodes in id order."""
        k, j, i = np.nonzero(self.node_active)
        return self.origin + np.stack([i, j, k], axis=1) * self.h

    def boundary_elements(self, f):
        """Indices (into the active element list) of elements touching outer face f."""
        axis, side = FACES[f]
        n_axis = (self.nx, self.ny, self.nz)[axis]
        target = 0 if side == 0 else n_axis - 1
        return np.nonzero(self.elem_ijk[:, axis] == target)[0]


def _element_dofs(mesh):
    nodes = mesh.elem_nodes                                   # (E, 8)
    return (3 * nodes[:, :, None] + np.arange(3)[None, None, :]).reshape(len(nodes), 24)


def assemble(prob, volume=True, abc=True):
    """Global system matrix (scipy CSR, complex128, scalar unknowns).

    Element contributions  (1/eps_e) Kc + s Kd - k0^2 mu_e Km  of every
    active element, plus  j k0 Mf + (j / 2 k0) Sf  on both tangential
    components of every active element face lying on an ABC outer face.
    Duplicates are summed by the COO -> CSR conversion."""
    mesh = Mesh(prob)
    N = mesh.n_unknowns
    rows, cols, vals = [], [], []
    eps = np.asarray(prob.eps_r, dtype=np.complex128).reshape(mesh.nz, mesh.ny, mesh.nx)
    mu = np.asarray(prob.mu_r, dtype=np.complex128).reshape(mesh.nz, mesh.ny, mesh.nx)
    ex, ey, ez = mesh.elem_ijk.T
    if volume and len(ex):
        Kc, Kd, Km = element_matrices(mesh.h)
        eps_e = eps[ez, ey, ex]
        mu_e = mu[ez, ey, ex]
        dofs = _element_dofs(mesh)
        ke = ((1.0 / eps_e)[:, None, None] * Kc[None] + prob.penalty_s * Kd[None]
              - (prob.k0 ** 2) * mu_e[:, None, None] * Km[None])
        rows.append(np.broadcast_to(dofs[:, :, None], ke.shape).ravel())
        cols.append(np.broadcast_to(dofs[:, None, :], ke.shape).ravel())
        vals.append(ke.ravel())
    if abc:
        for f in range(6):
            if prob.faces[f] != 0:
                continue
            axis, side = FACES[f]
            sel = mesh.boundary_elements(f)
            if len(sel) == 0:
                continue
            Mf, Sf = face_matrices(axis, mesh.h)
            kf = 1j * prob.k0 * Mf + (1j / (2.0 * prob.k0)) * Sf
            fnodes = mesh.elem_nodes[sel][:, face_local_nodes(axis, side)]    # (F, 4)
            for c in range(3):
                if c == axis:
                    continue
                d = 3 * fnodes + c
                rows.append(np.broadcast_to(d[:, :, None], (len(sel), 4, 4)).ravel())
                cols.append(np.broadcast_to(d[:, None, :], (len(sel), 4, 4)).ravel())
                vals.append(np.broadcast_to(kf[None], (len(sel), 4, 4)).ravel())
    if rows:
        r = np.concatenate(rows)
        c = np.concatenate(cols)
        v = np.concatenate(vals)
    else:
        r = c = np.zeros(0, dtype=np.int64)
        v = np.zeros(0, dtype=np.complex128)
    A = sp.coo_matrix((v, (r, c)), shape=(N, N)).tocsr()
    A.sum_duplicates()
    A = apply_constraints(A, constrained_unknowns(prob))
    A.sum_duplicates()
    return A


def penalty_surface_matrix(prob):
    """The penalty's surface integral as eq. (4) prints it (from eq. (2)),
    which the main reading drops.  In the standard operator sign used here
    it is  -s int_{S_ext + S_pec} (W . n)(div H) dS,  with S_ext the outer
    faces tagged ABC, S_pec the faces between an active and a PEC element,
    and n the outward normal of the active region; entry (3a + i, 3b + j) of
    one element face is  -s n_i int N_a dN_b/dx_j dS  (2x2 Gauss).  Not
    symmetric: the paper averages the system matrix with its transpose
    (section 3.1.4).  An oracle option, used to quantify that reading."""
    mesh = Mesh(prob)
    h = mesh.h
    s = prob.penalty_s
    pec = np.asarray(prob.pec).reshape(mesh.nz, mesh.ny, mesh.nx)
    n_el = (mesh.nx, mesh.ny, mesh.nz)
    rows, cols, vals = [], [], []
    dofs = _element_dofs(mesh)
    for f in range(6):
        axis, side = FACES[f]
        sgn = 1.0 if side else -1.0
        tang = [t for t in range(3) if t != axis]
        area = h[tang[0]] * h[tang[1]]
        F = np.zeros((24, 24))
        for w1, p1 in zip(GAUSS_WEIGHTS_UNIT, GAUSS_POINTS_UNIT):
            for w2, p2 in zip(GAUSS_WEIGHTS_UNIT, GAUSS_POINTS_UNIT):
                xi = np.zeros(3)
                xi[axis] = float(side)
                xi[tang[0]], xi[tang[1]] = p1, p2
                N, dN = volume_basis_at(xi, h)
                for a in range(8):
                    for b in range(8):
                        F[3 * a + axis, 3 * b:3 * b + 3] += -s * sgn * w1 * w2 * area * N[a] * dN[b]
        ijk = mesh.elem_ijk
        nb = ijk.copy()
        nb[:, axis] += 1 if side else -1
        outside = (nb[:, axis] < 0) | (nb[:, axis] >= n_el[axis])
        sel = outside & (prob.faces[f] == 0)
        inside = ~outside
        pec_nb = np.zeros(len(ijk), dtype=bool)
        pec_nb[inside] = pec[nb[inside, 2], nb[inside, 1], nb[inside, 0]] != 0
        sel |= pec_nb
        idx = np.nonzero(sel)[0]
        if len(idx) == 0:
            continue
        d = dofs[idx]
        rows.append(np.broadcast_to(d[:, :, None], (len(idx), 24, 24)).ravel())
        cols.append(np.broadcast_to(d[:, None, :], (len(idx), 24, 24)).ravel())
        vals.append(np.broadcast_to(F[None], (len(idx), 24, 24)).ravel())
    N = mesh.n_unknowns
    if not rows:
        return sp.csr_matrix((N, N), dtype=np.complex128)
    S = sp.coo_matrix((np.concatenate(vals).astype(np.complex128),
                       (np.concatenate(rows), np.concatenate(cols))), shape=(N, N)).tocsr()
    S.sum_duplicates()
    return S


def incident_field(wave, pts, k0):
    """H_i = p exp(-j k0 d.r) at points (m, 3) -> (m, 3) complex."""
    ph = np.exp(-1j * k0 * (pts @ np.asarray(wave.d, dtype=np.float64)))
    return ph[:, None] * np.asarray(wave.p, dtype=np.complex128)[None, :]


def rhs(prob, waves):
    """Right-hand sides (n_unknowns, nrhs) of eq. (4):
    sum over ABC faces of int N_a [ j k0 H_i,c - (n x curl H_i)_c ]
    + (j / 2 k0) int grad_t N_a . grad_t H_i,c   for tangential c,
    with curl H_i = -j k0 d x H_i and grad_t H_i,c = -j k0 d_t H_i,c."""
    mesh = Mesh(prob)
    k0 = prob.k0
    B = np.zeros((mesh.n_unknowns, len(waves)), dtype=np.complex128)
    for f in range(6):
        if prob.faces[f] != 0:
            continue
        axis, side = FACES[f]
        sel = mesh.boundary_elements(f)
        if len(sel) == 0:
            continue
        tang = [t for t in range(3) if t != axis]
        n = np.zeros(3)
        n[axis] = -1.0 if side == 0 else 1.0
        area = mesh.h[tang[0]] * mesh.h[tang[1]]
        fnodes = mesh.elem_nodes[sel][:, face_local_nodes(axis, side)]     # (F, 4)
        corner = mesh.origin + mesh.elem_ijk[sel] * mesh.h                  # (F, 3) element min corner
        for w1, p1 in zip(GAUSS_WEIGHTS_UNIT, GAUSS_POINTS_UNIT):
            for w2, p2 in zip(GAUSS_WEIGHTS_UNIT, GAUSS_POINTS_UNIT):
                w = w1 * w2 * area
                Nf, gt = face_basis_at((p1, p2), axis, side, mesh.h)       # (4,), (4, 3)
                local = np.zeros(3)
                local[axis] = side
                local[tang[0]], local[tang[1]] = p1, p2
                pts = corner + local * mesh.h                               # (F, 3)
                for r, wave in enumerate(waves):
                    d = np.asarray(wave.d, dtype=np.float64)
                    Hi = incident_field(wave, pts, k0)                      # (F, 3)
                    curlHi = -1j * k0 * np.cross(d[None, :], Hi)           # (F, 3)
                    ncurl = np.cross(n[None, :], curlHi)                    # (F, 3)
                    d_t = d.copy()
                    d_t[axis] = 0.0
                    for c in tang:
                        # j k0 N_a H_c - N_a (n x curl H_i)_c
                        term_m = (1j * k0 * Hi[:, c] - ncurl[:, c])[:, None] * Nf[None, :]
                        # (j / 2k0) grad_t N_a . grad_t H_c,  grad_t H_c = -j k0 d_t H_c
                        gradH = (-1j * k0) * Hi[:, c][:, None] * d_t[None, :]   # (F, 3)
                        term_s = (1j / (2.0 * k0)) * (gradH @ gt.T)              # (F, 4)
                        np.add.at(B[:, r], (3 * fnodes + c).ravel(), (w * (term_m + term_s)).ravel())
    B[constrained_unknowns(prob), :] = 0.0
    return B


def assemble_rows(prob, nodes):
    """Block rows of the global matrix for the given active node ids, each
    computed on its own by visiting the (at most 8) active elements that
    contain the node and the ABC element faces that contain it.

    Returns a dict node -> {neighbour node: 3x3 complex block}.  Used to check
    sampled rows of very large problems one by one."""
    mesh = Mesh(prob)
    Kc, Kd, Km = element_matrices(mesh.h)
    eps = np.asarray(prob.eps_r, dtype=np.complex128).reshape(mesh.nz, mesh.ny, mesh.nx)
    mu = np.asarray(prob.mu_r, dtype=np.complex128).reshape(mesh.nz, mesh.ny, mesh.nx)
    k, j, i = np.nonzero(mesh.node_active)
    out = {}
    face_mats = {axis: face_matrices(axis, mesh.h) for axis in range(3)}
    fixed = constrained_unknowns(prob).reshape(-1, 3)
    for node in nodes:
        node = int(node)
        gi, gj, gk = int(i[node]), int(j[node]), int(k[node])
        row = {}
        for la, (ax, ay, az) in enumerate(LOCAL_NODES):
            ex, ey, ez = gi - ax, gj - ay, gk - az
            if not (0 <= ex < mesh.nx and 0 <= ey < mesh.ny and 0 <= ez < mesh.nz):
                continue
            if not mesh.active_elem[ez, ey, ex]:
                continue
            ke = ((1.0 / eps[ez, ey, ex]) * Kc + prob.penalty_s * Kd
                  - prob.k0 ** 2 * mu[ez, ey, ex] * Km)
            for lb, (bx, by, bz) in enumerate(LOCAL_NODES):
                nb = int(mesh.node_id[ez + bz, ey + by, ex + bx])
                blk = row.setdefault(nb, np.zeros((3, 3), np.complex128))
                blk += ke[3 * la:3 * la + 3, 3 * lb:3 * lb + 3]
            # ABC faces of this element that contain the node
            for f in range(6):
                if prob.faces[f] != 0:
                    continue
                axis, side = FACES[f]
                eidx = (ex, ey, ez)[axis]
                n_axis = (mesh.nx, mesh.ny, mesh.nz)[axis]
                if eidx != (0 if side == 0 else n_axis - 1):
                    continue
                if (ax, ay, az)[axis] != side:
                    continue
                Mf, Sf = face_mats[axis]
                kf = 1j * prob.k0 * Mf + (1j / (2.0 * prob.k0)) * Sf
                fl = face_local_nodes(axis, side)
                pa = int(np.nonzero(fl == la)[0][0])
                for pb, lb in enumerate(fl):
                    bx, by, bz = LOCAL_NODES[lb]
                    nb = int(mesh.node_id[ez + bz, ey + by, ex + bx])
                    for c in range(3):
                        if c != axis:
                            row[nb][c, c] += kf[pa, pb]
        # symmetry-plane elimination: identity rows and columns
        for nb, blk in row.items():
            blk[fixed[node], :] = 0.0
            blk[:, fixed[nb]] = 0.0
            if nb == node:
                blk[fixed[node], fixed[node]] = 1.0
        out[node] = row
    return out


def scatter_to_grid(prob, x):
    """Nodal solution vector(s) (n_unknowns[, nrhs]) -> full grid
    (nrhs, nz+1, ny+1, nx+1, 3); nodes of no active element get 0."""
    mesh = Mesh(prob)
    x = np.asarray(x)
    if x.ndim == 1:
        x = x[:, None]
    nrhs = x.shape[1]
    out = np.zeros((nrhs, mesh.nz + 1, mesh.ny + 1, mesh.nx + 1, 3), dtype=np.complex128)
    for r in range(nrhs):
        out[r][mesh.node_active] = x[:, r].reshape(-1, 3)
    return out


def block_pattern(prob):
    """Block sparsity (row_ptr, col_idx) at node level implied by the scalar
    matrix: node b is a neighbour of node a when any scalar entry of the block
    (a, b) is stored by the assembly."""
    A = assemble(prob).tocoo()
    nb = Mesh(prob).n_nodes
    S = sp.coo_matrix((np.ones_like(A.row), (A.row // 3, A.col // 3)), shape=(nb, nb)).tocsr()
    S.sum_duplicates()
    S.sort_indices()
    return S.indptr.astype(np.int64), S.indices.astype(np.int64)


def to_bsr_blocks(A, row_ptr, col_idx):
    """Dense 3x3 blocks (nnzb, 3, 3) of scalar CSR matrix A on a block pattern."""
    A = A.tocsr()
    out = np.zeros((len(col_idx), 3, 3), dtype=np.complex128)
    rows = np.repeat(np.arange(len(row_ptr) - 1), np.diff(row_ptr))
    for i in range(3):
        for j in range(3):
            out[:, i, j] = np.asarray(A[3 * rows + i, 3 * col_idx + j]).ravel()
    return out
