"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed-form
1-D integrals, null spaces of the differential operators, conservation sums,
library direct solvers, the exact plane-wave solution of an empty box, and
the unknown counts the paper prints.  A plausible slip in the oracle (dropped
term, wrong sign, transposed index) fails at least one of them.
"""
import math
import os

import numpy as np
import scipy.sparse as sp
import pytest

import workloads as W
from oracle import fem, solve

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- closed forms
def _m1(a, b, h):
    return h / 6.0 * (2.0 if a == b else 1.0)


def _k1(a, b, h):
    return (1.0 if a == b else -1.0) / h


def _g1(a):
    # int N_a' N_b over [0, h] = -1/2 (a = 0) or +1/2 (a = 1), any b
    return -0.5 if a == 0 else 0.5


def _kron_tables(h):
    L = fem.LOCAL_NODES
    G = np.zeros((3, 3, 8, 8))
    M = np.zeros((8, 8))
    for a in range(8):
        for b in range(8):
            M[a, b] = np.prod([_m1(L[a, t], L[b, t], h[t]) for t in range(3)])
            for p in range(3):
                for q in range(3):
                    v = 1.0
                    for t in range(3):
                        if t == p and t == q:
                            v *= _k1(L[a, t], L[b, t], h[t])
                        elif t == p:
                            v *= _g1(L[a, t])
                        elif t == q:
                            v *= _g1(L[b, t])
                        else:
                            v *= _m1(L[a, t], L[b, t], h[t])
                    G[p, q, a, b] = v
    return G, M


@pytest.mark.parametrize("h", [(0.1, 0.1, 0.1), (0.1, 0.2, 0.35), (1.0, 0.5, 2.0)])
def test_element_tables_match_kronecker_closed_form(h):
    """2x2x2 Gauss is exact for these integrands, so the quadrature tables
    must equal the Kronecker products of the 1-D mass/stiffness/mixed
    integrals:  curl-curl = delta_ij sum_m G_mm - G_ji,  div-div = G_ij,
    mass = delta_ij M."""
    Kc, Kd, Km = fem.element_matrices(h)
    G, M = _kron_tables(h)
    scale = max(abs(Kc).max(), abs(Kd).max())
    for a in range(8):
        for b in range(8):
            for i in range(3):
                for j in range(3):
                    kc = (i == j) * sum(G[m, m, a, b] for m in range(3)) - G[j, i, a, b]
                    assert abs(Kc[3 * a + i, 3 * b + j] - kc) <= 1e-14 * scale
                    assert abs(Kd[3 * a + i, 3 * b + j] - G[i, j, a, b]) <= 1e-14 * scale
                    assert abs(Km[3 * a + i, 3 * b + j] - (i == j) * M[a, b]) <= 1e-15 * abs(Km).max()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_face_tables_match_closed_form(axis):
    h = (0.1, 0.2, 0.3)
    Mf, Sf = fem.face_matrices(axis, h)
    t1, t2 = [t for t in range(3) if t != axis]
    L = fem.LOCAL_NODES[fem.face_local_nodes(axis, 0)]
    for a in range(4):
        for b in range(4):
            m = _m1(L[a, t1], L[b, t1], h[t1]) * _m1(L[a, t2], L[b, t2], h[t2])
            s = (_k1(L[a, t1], L[b, t1], h[t1]) * _m1(L[a, t2], L[b, t2], h[t2])
                 + _m1(L[a, t1], L[b, t1], h[t1]) * _k1(L[a, t2], L[b, t2], h[t2]))
            assert abs(Mf[a, b] - m) <= 1e-16
            assert abs(Sf[a, b] - s) <= 1e-14 * abs(Sf).max()
    # tangential stiffness annihilates constants; face mass sums to the area
    assert abs(Sf.sum(axis=1)).max() <= 1e-14 * abs(Sf).max()
    assert abs(Mf.sum() - h[t1] * h[t2]) <= 1e-16


# ------------------------------------------------------------------ invariants
def _with(prob, **kw):
    import copy
    q = copy.deepcopy(prob)
    for k, v in kw.items():
        setattr(q, k, v)
    return q


def _field(mesh, fn):
    X = mesh.node_coords()
    return np.stack(fn(X[:, 0], X[:, 1], X[:, 2]), axis=1).astype(np.complex128).ravel()


def test_matrix_is_complex_symmetric():
    """Invariant (a): A = A^T (plain transpose), with lossy random eps/mu,
    PEC elements and ABC faces."""
    rng = np.random.default_rng(1)
    p = W.random_small(rng, n=(4, 3, 5), n_pec=3, lossy=True)
    p.mu_r[:] = rng.uniform(1.0, 2.0, size=p.mu_r.shape)
    A = fem.assemble(p)
    assert abs(A - A.T).max() <= 1e-14 * abs(A).max()
    # and it is not Hermitian: the ABC and the loss make it complex
    assert abs(A - A.conj().T).max() > 1e-3 * abs(A).max()


def test_curl_and_penalty_null_spaces():
    """Invariant (b): the volume curl-curl + penalty part annihilates constant
    fields; the curl part alone annihilates gradient fields that the
    trilinear space represents exactly; the penalty part alone annihilates
    divergence-free fields represented exactly.  Heterogeneous eps and PEC
    holes must not matter."""
    rng = np.random.default_rng(2)
    p = W.random_small(rng, n=(4, 4, 4), n_pec=2, lossy=True,
                       faces=(W.FACE_NATURAL,) * 6)
    p.origin = (0.3, -0.2, 0.1)
    mesh = fem.Mesh(p)
    K = fem.assemble(_with(p, k0=0.0, penalty_s=1.0))        # curl + penalty
    C = fem.assemble(_with(p, k0=0.0, penalty_s=0.0))        # curl only
    P = K - C                                                # penalty only
    scale = abs(K).max()
    for c in range(3):
        e = np.zeros(mesh.n_unknowns, np.complex128)
        e[c::3] = 1.0
        assert abs(K @ e).max() <= 1e-13 * scale
    grads = [lambda x, y, z: (np.ones_like(x), 0 * x, 0 * x),
             lambda x, y, z: (y, x, 0 * x),                 # grad(xy)
             lambda x, y, z: (y * z, x * z, x * y),         # grad(xyz)
             lambda x, y, z: (2 * x, 2 * y, 0 * z)]         # grad(x^2 + y^2)
    for g in grads:
        v = _field(mesh, g)
        assert abs(C @ v).max() <= 1e-12 * scale * abs(v).max()
    divfree = [lambda x, y, z: (y, z, x),
               lambda x, y, z: (y * z, x * z, 0 * z),       # div = 0
               lambda x, y, z: (z, 0 * x, y)]
    for g in divfree:
        v = _field(mesh, g)
        assert abs(P @ v).max() <= 1e-12 * scale * abs(v).max()
    # the curl part does NOT annihilate a rotational field: guards against a
    # vanished operator passing the checks above
    v = _field(mesh, lambda x, y, z: (-y, x, 0 * z))
    assert abs(C @ v).max() > 1e-3 * scale * abs(v).max()


def test_mass_sums_to_volume():
    """Invariant (c): for each component the k0^2 mu mass part sums to
    k0^2 * sum_e mu_e V_e over the active elements."""
    rng = np.random.default_rng(3)
    p = W.random_small(rng, n=(3, 4, 2), n_pec=2, faces=(W.FACE_NATURAL,) * 6,
                       h=(0.1, 0.15, 0.2))
    p.mu_r[:] = rng.uniform(1.0, 3.0, size=p.mu_r.shape) + 0.1j
    k0 = 2.7
    Mk = fem.assemble(_with(p, k0=0.0)) - fem.assemble(_with(p, k0=k0))   # = k0^2 mu M
    V = p.h[0] * p.h[1] * p.h[2]
    expected = k0 ** 2 * V * p.mu_r[p.pec == 0].sum()
    for c in range(3):
        sub = Mk[c::3, :][:, c::3]
        assert abs(sub.sum() - expected) <= 1e-13 * abs(expected)
        # no coupling between different components
        other = Mk[c::3, :][:, (c + 1) % 3::3]
        assert abs(other).max() <= 1e-16 * abs(expected)


def test_interior_stencil_closed_form():
    """Free space, s = 1, eps = mu = 1: curl-curl + grad-div is the vector
    Laplacian, so an interior block row is diagonal and each component sees
    the Kronecker stencil  K(x)M(x)M + M(x)K(x)M + M(x)M(x)K - k0^2 M(x)M(x)M
    with 1-D K = (1/h) [-1, 2, -1] and M = (h/6) [1, 4, 1]."""
    n = 4
    p, _ = W.free_cube(n, wavelengths=0.4)
    h = p.h[0]
    k0 = p.k0
    p.faces = (W.FACE_NATURAL,) * 6
    A = fem.assemble(p)
    mesh = fem.Mesh(p)
    K1 = {-1: -1 / h, 0: 2 / h, 1: -1 / h}
    M1 = {-1: h / 6, 0: 4 * h / 6, 1: h / 6}
    i0 = j0 = k0i = 2
    a = mesh.node_id[k0i, j0, i0]
    centre = None
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                b = mesh.node_id[k0i + dz, j0 + dy, i0 + dx]
                val = (K1[dx] * M1[dy] * M1[dz] + M1[dx] * K1[dy] * M1[dz]
                       + M1[dx] * M1[dy] * K1[dz] - k0 ** 2 * M1[dx] * M1[dy] * M1[dz])
                blk = A[3 * a:3 * a + 3, 3 * b:3 * b + 3].toarray()
                assert np.allclose(blk, val * np.eye(3), rtol=0, atol=1e-14 * 3 / h)
                if dx == dy == dz == 0:
                    centre = blk[0, 0]
    assert abs(centre - (8 * h / 3 - k0 ** 2 * 8 * h ** 3 / 27)) <= 1e-14 * 8 * h / 3
    # one scalar row touches 27 nodes, one component each (other stored
    # entries of the 3x3 blocks cancel to rounding)
    row = A[3 * a].toarray().ravel()
    assert (abs(row) > 1e-12 / h).sum() == 27


def test_abc_row_sums():
    """The ABC adds j k0 Mf + (j / 2 k0) Sf on the tangential components
    only.  Sf annihilates constants, so each tangential row sum of the
    added part is j k0 times the node's share of face area (h^2 / 4 per
    incident quad); the normal component gets nothing."""
    n = 3
    p, _ = W.free_cube(n)
    h = p.h[0]
    base = fem.assemble(_with(p, faces=(W.FACE_NATURAL,) * 6))
    for f in range(6):
        faces = [W.FACE_NATURAL] * 6
        faces[f] = W.FACE_ABC
        D = fem.assemble(_with(p, faces=tuple(faces))) - base
        axis, side = fem.FACES[f]
        mesh = fem.Mesh(p)
        idx = [slice(None)] * 3
        idx[2 - axis] = 0 if side == 0 else -1            # node_id is (z, y, x)
        face_nodes = mesh.node_id[tuple(idx)]
        counts = np.zeros(face_nodes.shape)
        # number of face quads incident to each face node
        for t in range(2):
            sl = [slice(None)] * 2
            for u in range(2):
                s2 = [slice(0, -1), slice(0, -1)]
                s2[0] = slice(t, counts.shape[0] - 1 + t)
                s2[1] = slice(u, counts.shape[1] - 1 + u)
                counts[tuple(s2)] += 1
        for c in range(3):
            rows = 3 * face_nodes.ravel() + c
            rs = np.asarray(D[rows, :].sum(axis=1)).ravel()
            if c == axis:
                assert abs(rs).max() == 0.0
                assert D[rows, :].nnz == 0 or abs(D[rows, :]).max() == 0.0
            else:
                assert np.allclose(rs, 1j * p.k0 * counts.ravel() * h * h / 4, rtol=1e-13, atol=0)
        interior = np.setdiff1d(np.arange(mesh.n_nodes), face_nodes.ravel())
        assert abs(D[np.concatenate([3 * interior + c for c in range(3)]), :]).max() == 0.0
        # diagonal of a node inside the face (4 quads): face mass 4 (h/3)^2,
        # tangential stiffness 4 * 2/3; coefficients j k0 and + j / (2 k0) of eq. (3)
        a = face_nodes[1, 1]
        t = [u for u in range(3) if u != axis][0]
        want = 1j * p.k0 * 4 * h * h / 9 + (1j / (2 * p.k0)) * 4 * (2.0 / 3.0)
        assert abs(D[3 * a + t, 3 * a + t] - want) <= 1e-14 * abs(want)


def test_rhs_normal_incidence_closed_form():
    """Wave along +z, polarised along x, ABC box.  On the -z face (incoming)
    n x curl H_i = -j k0 H_i, so interior nodes of that face get
    b_x = 2 j k0 (4 h^2 / 4); on the +z face (outgoing) g(H_i) equals
    n x curl H_i and b = 0; nodes off the boundary get 0."""
    n = 4
    p, waves = W.free_cube(n)
    h = p.h[0]
    b = fem.rhs(p, waves)[:, 0].reshape(-1, 3)
    mesh = fem.Mesh(p)
    inner = mesh.node_id[0, 1:-1, 1:-1].ravel()
    assert np.allclose(b[inner, 0], 2j * p.k0 * h * h, rtol=1e-14, atol=0)
    assert abs(b[inner, 1:]).max() == 0.0
    outer = mesh.node_id[-1, 1:-1, 1:-1].ravel()
    assert abs(b[outer]).max() <= 1e-14 * p.k0 * h * h
    interior = mesh.node_id[1:-1, 1:-1, 1:-1].ravel()
    assert abs(b[interior]).max() == 0.0


def test_rhs_side_face_sums():
    """Same wave; on the +x face (n = +x), -(n x curl H_i)_z = j k0 H_x, the
    tangential field H_y = H_z = 0, so the z-rows of that face sum to
    j k0 int exp(-j k0 z) dS (partition of unity).  Compared with the exact
    integral within the 2-point Gauss error."""
    p, waves = W.free_cube(7, wavelengths=0.7)   # the integral is not zero
    p.faces = (W.FACE_NATURAL, W.FACE_ABC) + (W.FACE_NATURAL,) * 4
    b = fem.rhs(p, waves)[:, 0].reshape(-1, 3)
    mesh = fem.Mesh(p)
    L = p.nz * p.h[2]
    Ly = p.ny * p.h[1]
    face = mesh.node_id[:, :, -1].ravel()
    exact = 1j * p.k0 * Ly * (1 - np.exp(-1j * p.k0 * L)) / (1j * p.k0)
    got = b[face, 2].sum()
    assert abs(got - exact) <= 1e-3 * abs(exact)
    assert abs(b[face, :2]).max() == 0.0


# ------------------------------------------------------------------ the solve
@pytest.mark.parametrize("n", [(2, 2, 2), (3, 3, 3), (4, 3, 4)])
def test_dense_sparse_cocg_agree(n):
    """Invariant (d): LAPACK LU, SuperLU and COCG-Jacobi give the same
    solution on tiny random meshes with one PEC element."""
    rng = np.random.default_rng(sum(n))
    p = W.random_small(rng, n=n, n_pec=1, lossy=False)
    waves = [W.random_wave(rng) for _ in range(2)]
    A = fem.assemble(p)
    B = fem.rhs(p, waves)
    x_dense = solve.dense_solve(A, B)
    x_sparse = solve.sparse_solve(A, B)
    assert np.linalg.norm(x_dense - x_sparse) <= 1e-12 * np.linalg.norm(x_dense)
    for r in range(2):
        res = solve.cocg(A, B[:, r], rtol=1e-14, maxiter=5000)
        assert not res.breakdown
        assert solve.residual(A, res.x, B[:, r]) <= 1e-13
        assert np.linalg.norm(res.x - x_dense[:, r]) <= 1e-10 * np.linalg.norm(x_dense[:, r])


def test_empty_box_reproduces_incident_wave():
    """Invariant (e): with no scatterer the total field is the incident
    plane wave.  The nodal error is a few percent at 10 nodes per
    wavelength and falls about 4x (second order) when h halves.  The
    opposite right-hand-side sign gives an O(1) error."""
    errs = []
    for n in (10, 20):
        p, waves = W.free_cube(n)
        A = fem.assemble(p)
        b = fem.rhs(p, waves)[:, 0]
        res = solve.cocg(A, b, rtol=1e-11, maxiter=5000)
        hi = fem.incident_field(waves[0], fem.Mesh(p).node_coords(), p.k0).ravel()
        errs.append(np.linalg.norm(res.x - hi) / np.linalg.norm(hi))
        if n == 10:
            wrong = solve.cocg(A, -b, rtol=1e-11, maxiter=5000)
            assert np.linalg.norm(wrong.x - hi) / np.linalg.norm(hi) > 1.0
    assert 0.01 < errs[0] < 0.1
    assert errs[0] / errs[1] > 3.0


def test_oblique_wave_in_lossy_free_box_converges():
    """The empty-box property must hold for any direction/polarisation (all
    six faces then carry incoming and outgoing parts) and for mesh sizes that
    are not a whole number of wavelengths."""
    rng = np.random.default_rng(5)
    wave = W.random_wave(rng)
    errs = []
    for n in (7, 14):
        p, _ = W.free_cube(n, wavelengths=0.7)
        A = fem.assemble(p)
        b = fem.rhs(p, [wave])[:, 0]
        x = solve.cocg(A, b, rtol=1e-11, maxiter=5000).x
        hi = fem.incident_field(wave, fem.Mesh(p).node_coords(), p.k0).ravel()
        errs.append(np.linalg.norm(x - hi) / np.linalg.norm(hi))
    assert errs[0] < 0.1 and errs[0] / errs[1] > 3.0


def test_cocg_breakdown_detected():
    """b with b^T D^-1 b = 0 makes rho_0 = 0: COCG must report breakdown."""
    p, _ = W.free_cube(3)
    A = fem.assemble(p)
    D = A.diagonal()
    v = np.zeros(A.shape[0], np.complex128)
    v[0], v[1] = 1.0, 1.0j
    b = v * np.sqrt(D)
    assert abs(solve.bilinear(b, b / D)) < 1e-15
    res = solve.cocg(A, b, rtol=1e-10, maxiter=100)
    assert res.breakdown and res.iters == 0


# ----------------------------------------------------------- bookkeeping pins
def _golden_rows(name):
    rows = []
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append([int(t) for t in line.split()[:2]])
    return rows


def test_unknown_counts_match_paper():
    """Three complex unknowns per node, six real degrees of freedom per node:
    the paper's printed counts (section 1, figure 3, section 3.2)."""
    rows = _golden_rows("paper_sizes.txt")
    nodes_per_side, unknowns = rows[0]
    m = nodes_per_side - 1
    p = W._blank(m, m, m, (0.1,) * 3, (0, 0, 0), 2 * math.pi)
    assert fem.Mesh(p).n_unknowns == unknowns
    for nodes, dof in rows[1:]:
        assert 2 * 3 * nodes == dof


def test_pec_removes_only_interior_nodes():
    """PEC elements are removed; nodes on the PEC surface stay active."""
    p, _ = W.pec_cube(30)
    mesh = fem.Mesh(p)
    assert int(p.pec.sum()) == 1000
    assert mesh.n_nodes == 31 ** 3 - 9 ** 3


def test_row_sampler_matches_global_assembly():
    """The one-row-at-a-time assembly used to check huge problems agrees
    with the global COO assembly on a small random problem."""
    rng = np.random.default_rng(7)
    p = W.random_small(rng, n=(4, 3, 3), n_pec=3, lossy=True)
    p.mu_r[:] = 1.0 + rng.uniform(0, 1, size=p.mu_r.shape)
    A = fem.assemble(p)
    mesh = fem.Mesh(p)
    nodes = rng.choice(mesh.n_nodes, size=12, replace=False)
    rows = fem.assemble_rows(p, nodes)
    for a in nodes:
        full = A[3 * a:3 * a + 3].toarray()
        got = np.zeros_like(full)
        for b, blk in rows[a].items():
            got[:, 3 * b:3 * b + 3] = blk
        assert np.abs(got - full).max() <= 1e-14 * abs(A).max()


# ------------------------------------------------------------ symmetry planes
@pytest.mark.parametrize("cut_x,cut_y", [(True, False), (False, True), (True, True)])
def test_symmetry_planes_reproduce_the_whole_box(cut_x, cut_y):
    """Section 3.1.3: a mirror-symmetric box (PEC cube at the centre, x-polarised
    wave along +z) solved on its x >= 0 half with n x H = 0 on x = 0 (eq. (6b)),
    and/or its y >= 0 half with n . H = 0 on y = 0 (eq. (6a)), gives exactly the
    whole box's nodal field there (direct solves on both).  Constraining the
    wrong components, or dropping the elimination, breaks the equality."""
    n = 8
    full, waves = W.mirrored_pec_cube(n)
    cut, _ = W.mirrored_pec_cube(n, cut_x=cut_x, cut_y=cut_y)
    Hf = fem.scatter_to_grid(full, solve.sparse_solve(fem.assemble(full), fem.rhs(full, waves)))[0]
    Hc = fem.scatter_to_grid(cut, solve.sparse_solve(fem.assemble(cut), fem.rhs(cut, waves)))[0]
    x0 = n // 2 if cut_x else 0
    y0 = n // 2 if cut_y else 0
    ref = Hf[:, y0:, x0:, :]
    scale = np.abs(Hf).max()
    assert np.abs(Hc - ref).max() <= 1e-10 * scale
    # the whole box's field obeys the plane conditions by itself
    mid = n // 2
    assert np.abs(Hf[:, :, mid, 1:]).max() <= 1e-10 * scale      # x = 0: H_y = H_z = 0
    assert np.abs(Hf[:, mid, :, 1]).max() <= 1e-10 * scale       # y = 0: H_y = 0
    assert np.abs(Hf[:, :, mid, 0]).max() > 1e-3 * scale         # H_x is free on x = 0


def test_symmetry_plane_elimination_keeps_identity_rows():
    """The fixed unknowns' rows and columns are those of the identity, their
    right-hand side is zero, and the matrix stays complex-symmetric; an
    antisymmetry face fixes the two tangential components and a symmetry
    face the normal one."""
    p, waves = W.mirrored_pec_cube(6, cut_x=True, cut_y=True)
    A = fem.assemble(p).tocsr()
    B = fem.rhs(p, waves)
    C = fem.constrained_unknowns(p)
    m = fem.Mesh(p)
    k, j, i = np.nonzero(m.node_active)
    on_x, on_y = i == 0, j == 0
    expect = np.zeros((m.n_nodes, 3), bool)
    expect[on_x, 1] = expect[on_x, 2] = True
    expect[on_y, 1] = True
    assert np.array_equal(C, expect.ravel())
    idx = np.nonzero(C)[0]
    sub = A[idx]
    assert np.array_equal(sub.toarray(), np.eye(A.shape[0])[idx])
    assert abs(A[:, idx] - sp_eye_cols(A.shape[0], idx)).max() == 0.0
    assert np.all(B[idx] == 0)
    assert abs(A - A.T).max() <= 1e-14 * abs(A).max()


def sp_eye_cols(n, idx):
    import scipy.sparse as sp
    return sp.identity(n, dtype=np.complex128, format="csc")[:, idx]


def test_row_sampler_applies_symmetry_planes():
    """The one-row-at-a-time assembly applies the same elimination as the
    global one."""
    p, _ = W.mirrored_pec_cube(6, cut_x=True, cut_y=True)
    A = fem.assemble(p).tocsr()
    m = fem.Mesh(p)
    nodes = np.arange(0, m.n_nodes, 7)
    rows = fem.assemble_rows(p, nodes)
    for a in nodes:
        for b, blk in rows[int(a)].items():
            ref = A[3 * int(a):3 * int(a) + 3, 3 * b:3 * b + 3].toarray()
            assert np.allclose(blk, ref, rtol=0, atol=1e-13 * abs(A).max())


# ---------------------------------------- the printed penalty surface term
def test_penalty_surface_term_closed_form():
    """The literal surface term -s int (W.n)(div H) dS applied to the nodal
    interpolant of a constant field is zero (div H = 0).  Applied to
    H = (x, 0, 0) (div H = 1) it gives -s n_k int N_a dS in row (a, k), so
    the k rows summed over the nodes of the face normal to axis k on side
    +/- give -/+ s times that face's area (partition of unity), and the k
    rows of nodes on neither of those two faces are zero."""
    p, _ = W.free_cube(4)
    p.h = (0.1, 0.15, 0.2)
    p.penalty_s = 0.7
    S = fem.penalty_surface_matrix(p)
    m = fem.Mesh(p)
    xyz = m.node_coords()
    const = np.tile(np.array([1.0, -2.0, 0.5]), m.n_nodes)
    assert np.abs(S @ const).max() <= 1e-13
    hx = np.zeros((m.n_nodes, 3))
    hx[:, 0] = xyz[:, 0]
    y = (S @ hx.ravel()).reshape(-1, 3)
    ext = np.array([p.nx * p.h[0], p.ny * p.h[1], p.nz * p.h[2]])
    for k in range(3):
        t = [a for a in range(3) if a != k]
        area = ext[t[0]] * ext[t[1]]
        on_plus = np.isclose(xyz[:, k], ext[k])
        on_minus = np.isclose(xyz[:, k], 0.0)
        assert abs(y[on_plus, k].sum() - (-p.penalty_s * area)) <= 1e-12
        assert abs(y[on_minus, k].sum() - (+p.penalty_s * area)) <= 1e-12
        assert np.abs(y[~(on_plus | on_minus), k]).max() <= 1e-13


def test_printed_penalty_term_with_symmetrisation_breaks_the_empty_box():
    """Reading A3 (surface term dropped, matrix symmetric) reproduces the
    incident wave in an empty ABC box to discretisation error; keeping the
    printed surface term does too (it vanishes on divergence-free fields);
    but averaging that matrix with its transpose, as section 3.1.4 does, adds
    -s int (div W)(H.n) dS, which does not vanish on H_i, and the solution no
    longer resembles it (measured: 4.8 %, 6.4 % and 90 % at 10^3)."""
    p, waves = W.free_cube(10)
    A = fem.assemble(p)
    b = fem.rhs(p, waves)[:, 0]
    S = fem.penalty_surface_matrix(p)
    Hi = fem.incident_field(waves[0], fem.Mesh(p).node_coords(), p.k0).ravel()

    def err(M):
        x = solve.sparse_solve(M.tocsc(), b)
        return np.linalg.norm(x - Hi) / np.linalg.norm(Hi)

    e_a3, e_lit = err(A), err(A + S)
    e_sym = err(((A + S) + (A + S).T) / 2)
    assert e_a3 < 0.06 and e_lit < 0.1
    assert e_sym > 0.5


def test_condition_estimate_brackets_the_exact_condition_number():
    """The Hager-Higham estimate is a lower bound of ||A||_1 ||A^-1||_1 and,
    on these small systems, within a factor 10 of it, also from the
    shared-factorisation variant, whose solution is the dense one."""
    rng = np.random.default_rng(12)
    for _ in range(3):
        p = W.random_small(rng, n=(3, 3, 2), n_pec=1, lossy=True)
        A = fem.assemble(p)
        exact = float(abs(np.linalg.cond(A.toarray(), 1)))
        est = solve.condest(A)
        assert exact / 10.0 <= est <= exact * (1 + 1e-10), (est, exact)
        b = fem.rhs(p, [W.random_wave(rng)])[:, 0]
        x, est2 = solve.lu_solve_condest(A, b)   # the estimator draws its own start vectors
        assert exact / 10.0 <= est2 <= exact * (1 + 1e-10), (est2, exact)
        xd = solve.dense_solve(A, b)
        assert np.linalg.norm(x - xd) <= 1e-12 * np.linalg.norm(xd)


def test_bsr_blocks_and_grid_scatter_are_lossless():
    """to_bsr_blocks cuts the scalar matrix into the 3x3 blocks of the block
    pattern with nothing left over (the blocks reassemble A exactly), and
    scatter_to_grid puts every unknown at its node and zeros elsewhere."""
    import scipy.sparse as sp

    rng = np.random.default_rng(13)
    p = W.random_small(rng, n=(4, 3, 3), n_pec=3)
    A = fem.assemble(p)
    rp, ci = fem.block_pattern(p)
    blocks = fem.to_bsr_blocks(A, rp, ci)
    B = sp.bsr_matrix((blocks, ci, rp), shape=A.shape).tocsr()
    assert abs(B - A).max() == 0.0
    mesh = fem.Mesh(p)
    x = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    H = fem.scatter_to_grid(p, x)
    assert H.shape == (1, p.nz + 1, p.ny + 1, p.nx + 1, 3)
    np.testing.assert_array_equal(H[0][mesh.node_active].reshape(-1), x)
    assert np.all(H[0][~mesh.node_active] == 0)


def test_bic0_on_a_full_pattern_is_the_complex_symmetric_cholesky_factor():
    """With every entry in the pattern, eq. (5)'s incomplete factor is the
    exact complex-symmetric Cholesky factor: L L^T (not L L^H) = A."""
    rng = np.random.default_rng(3)
    n = 12
    M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = M @ M.T + 10 * n * np.eye(n)
    L = solve.bic0_factor(sp.csr_matrix(A), n // 3).toarray()
    assert np.all(np.triu(L, 1) == 0)
    np.testing.assert_allclose(L @ L.T, A, rtol=0, atol=1e-12 * abs(A).max())
    assert np.all(np.diag(L).real > 0)           # principal square roots
    assert abs(L @ L.conj().T - A).max() > 1e-3 * abs(A).max()


@pytest.mark.parametrize("nodes_per_block", [1, 8, 64])
def test_bic0_is_exact_on_its_pattern_and_stays_inside_blocks(nodes_per_block):
    """Incomplete Cholesky's defining property: (L L^T)_ij = a_ij at every
    stored (i, j) inside a block; L has no entry outside the blocks of B
    consecutive nodes and none above the diagonal.  B = 1 keeps only each
    node's 3x3 diagonal block, whose factor is then exact."""
    p, _ = W.pec_sphere_shell(n=6, radius=0.15, shell=0.06, seed=2)
    A = fem.assemble(p).tocsr()
    L = solve.bic0_factor(A, nodes_per_block)
    size = 3 * nodes_per_block
    Lc = L.tocoo()
    assert np.all(Lc.row // size == Lc.col // size) and np.all(Lc.row >= Lc.col)
    S = A.copy()
    S.data = np.ones_like(S.data)
    Sc = S.tocoo()
    inside = Sc.row // size == Sc.col // size
    LL = (L @ L.T).tocsr()
    diff = np.asarray(LL[Sc.row[inside], Sc.col[inside]]).ravel() - np.asarray(A[Sc.row[inside], Sc.col[inside]]).ravel()
    assert abs(diff).max() <= 1e-13 * abs(A).max()
    assert L.nnz == (np.count_nonzero(inside) + A.shape[0]) // 2


def test_bic0_apply_solves_with_l_lt_and_pcocg_reaches_the_lu_solution():
    p, w = W.pec_sphere_shell(n=6, radius=0.15, shell=0.06, seed=2)
    A = fem.assemble(p).tocsr()
    b = fem.rhs(p, w)[:, 0]
    L = solve.bic0_factor(A, 16)
    rng = np.random.default_rng(5)
    r = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    z = solve.bic0_apply(L, r)
    assert np.linalg.norm((L @ (L.T @ z)) - r) <= 1e-12 * np.linalg.norm(r)
    res = solve.pcocg(A, b, lambda v: solve.bic0_apply(L, v), rtol=1e-12, maxiter=2000)
    x = solve.dense_solve(A, b)
    assert not res.breakdown and res.rel_res <= 1e-12
    assert np.linalg.norm(res.x - x) <= 1e-9 * np.linalg.norm(x)
    # the same recurrence with Jacobi is the oracle's COCG, iterate for iterate
    d = 1.0 / A.diagonal()
    a = solve.pcocg(A, b, lambda v: d * v, rtol=1e-10, maxiter=2000)
    c = solve.cocg(A, b, rtol=1e-10, maxiter=2000)
    assert a.iters == c.iters and np.array_equal(a.x, c.x)
