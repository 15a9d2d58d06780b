"""Seeded synthetic inputs shaped like the paper's workloads.

This module only synthesises meshes and coefficient data. It holds none of the
integration method's arithmetic (no shape functions, Jacobians or quadrature
sums) and is shared by the GPU path's callers and by the CPU oracle's tests, so
that both consume exactly the same arrays.

The paper measures per-element kernels on meshes whose size it states only as
"more than 1e5 elements per subdomain" (Sec. 3.1) and publishes no data set, so
these generators stand in for its inputs: jittered structured meshes of affine
tetrahedra and of 6-node prisms, and coefficient sets of the two kinds Sec. 4.1
describes ("Poisson": Laplacian plus a right-hand side, and "conv-diff": all
twenty coefficients).

Array layouts (all C-contiguous NumPy arrays):

* ``coords``: structure-of-arrays, shape ``(n_vert * 3, n_elem)``; row
  ``v * 3 + d`` holds coordinate ``d`` of local vertex ``v`` for every element.
* compact coefficients, per element: shape ``(n_slots, n_elem)``; per
  quadrature point: shape ``(n_slots * n_q, n_elem)`` with row ``j * n_q + q``.
  Slot numbering for scalar problems follows the coefficient indices of the
  generic algorithm (Algorithm 1): slot ``4 * a + b`` is ``c[a][b]`` and slot
  ``16 + a`` is ``d[a]``, index 0 being the function value and 1..3 the x, y, z
  derivatives. For elasticity the slots are ``(E, nu, f_x, f_y, f_z)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Kuhn subdivision of a cube into 6 tetrahedra: one tetrahedron per permutation
# of the three axes, in lexicographic order, with the parity of each
# permutation (odd ones get two vertices swapped so that all have the same
# orientation as the reference tetrahedron).
_KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))
_KUHN_ODD = (False, True, True, False, False, True)


@dataclass
class Mesh:
    """A mesh with per-element duplicated vertex coordinates.

    ``coords`` is the SoA array described in the module docstring; ``nodes``
    (n_nodes, 3) and ``conn`` (n_elem, n_vert) give the conforming node
    numbering, used only by tests that assemble (patch test)."""

    elem: str            # "tet4" or "prism6"
    coords: np.ndarray   # (n_vert*3, n_elem) float64
    nodes: np.ndarray    # (n_nodes, 3) float64
    conn: np.ndarray     # (n_elem, n_vert) int64
    boundary: np.ndarray  # (n_nodes,) bool, node lies on the domain boundary

    @property
    def n_elem(self) -> int:
        return int(self.coords.shape[1])


def _soa(nodes: np.ndarray, conn: np.ndarray) -> np.ndarray:
    """Gather per-element vertex coordinates into the SoA layout."""
    n_elem, n_vert = conn.shape
    out = np.empty((n_vert * 3, n_elem), dtype=np.float64)
    for v in range(n_vert):
        for d in range(3):
            out[v * 3 + d] = nodes[conn[:, v], d]
    return out


def _morton_keys(points: np.ndarray, bits: int = 10) -> np.ndarray:
    """Z-order (Morton) keys of points quantised to 2^bits cells per axis of
    their bounding box."""
    lo = points.min(axis=0)
    span = np.maximum(points.max(axis=0) - lo, 1e-300)
    q = np.minimum(((points - lo) / span * (1 << bits)).astype(np.int64), (1 << bits) - 1)
    key = np.zeros(points.shape[0], dtype=np.int64)
    for b in range(bits):
        for d in range(3):
            key |= ((q[:, d] >> b) & 1) << (3 * b + d)
    return key


def morton_order(mesh: Mesh) -> tuple[Mesh, np.ndarray]:
    """The same mesh with nodes renumbered and elements reordered along a
    Z-order curve (nodes by position, elements by centroid), so that elements
    close in the element order touch nodes close in memory. Returns the new
    mesh and the element permutation (new element i is old element perm[i])
    for reordering per-element data."""
    node_perm = np.argsort(_morton_keys(mesh.nodes), kind="stable")
    new_id = np.empty_like(node_perm)
    new_id[node_perm] = np.arange(node_perm.size)
    nodes = np.ascontiguousarray(mesh.nodes[node_perm])
    conn = new_id[mesh.conn]
    perm = np.argsort(_morton_keys(nodes[conn].mean(axis=1)), kind="stable")
    conn = np.ascontiguousarray(conn[perm])
    return Mesh(mesh.elem, _soa(nodes, conn), nodes, conn, mesh.boundary[node_perm]), perm


def tet_cube(N: int, seed: int | np.random.Generator, jitter: float = 0.1) -> Mesh:
    """Unit cube as N^3 cells, each split into 6 Kuhn tetrahedra (6 N^3 elements).

    Nodes (i, j, k) are numbered with i fastest. Interior nodes move by
    ``U(-jitter, jitter) * h`` in each coordinate (boundary nodes stay put), the
    first draw of ``seed``'s stream. Element ``6 * (i + N * (j + N * k)) + t``
    is tetrahedron ``t`` of cell (i, j, k); its vertices are the cell's low
    corner, then one step along each axis of permutation ``t`` in turn, with
    local vertices 1 and 2 swapped for odd permutations so every element has
    positive orientation."""
    rng = seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)
    if N < 1:
        raise ValueError("N must be >= 1")
    h = 1.0 / N
    n1 = N + 1
    kk, jj, ii = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(n1), indexing="ij")
    ijk = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1).astype(np.int64)
    U = rng.uniform(-jitter, jitter, (n1 ** 3, 3))
    boundary = np.any((ijk == 0) | (ijk == N), axis=1)
    U[boundary] = 0.0
    nodes = ijk * h + U * h

    def nid(i, j, k):
        return i + n1 * (j + n1 * k)

    ck, cj, ci = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    cell = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1).astype(np.int64)  # cell id order
    n_cell = cell.shape[0]
    conn = np.empty((n_cell, 6, 4), dtype=np.int64)
    for t, perm in enumerate(_KUHN_PERMS):
        p = cell.copy()
        verts = [nid(p[:, 0], p[:, 1], p[:, 2])]
        for ax in perm:
            p[:, ax] += 1
            verts.append(nid(p[:, 0], p[:, 1], p[:, 2]))
        if _KUHN_ODD[t]:
            verts[1], verts[2] = verts[2], verts[1]
        conn[:, t, :] = np.stack(verts, axis=1)
    conn = conn.reshape(n_cell * 6, 4)
    return Mesh("tet4", _soa(nodes, conn), nodes, conn, boundary)


def prism_layers(n: int, L: int, seed: int | np.random.Generator, jitter: float = 0.1,
                 sliver: bool = True, sliver_ratio: float = 1e-3) -> Mesh:
    """Unit cube as an n x n triangulated grid extruded through L layers.

    Each xy square (i, j) is split along its (0,0)-(1,1) diagonal into two
    triangles t = 0, 1; element ``2 * (i + n * j) + t + 2 n^2 * layer`` is the
    prism over triangle t in that layer, with bottom vertices 0-2 and top vertex
    ``v + 3`` above bottom vertex ``v``.

    With ``sliver`` (needs L >= 2) layer ``L // 2`` has thickness
    ``h_xy * sliver_ratio``; the other layers share the rest of the unit height.
    The two node levels bounding the sliver carry the same xy jitter (no
    lateral shear through the thin layer). Interior nodes move by
    ``U(-jitter, jitter) * h_xy`` in x and y and by ``U(-jitter, jitter)`` times
    the thinner adjacent layer in z, so faces are non-planar and the elements
    are not affine. Boundary nodes stay put."""
    rng = seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)
    if n < 1 or L < 1:
        raise ValueError("n and L must be >= 1")
    if sliver and L < 2:
        raise ValueError("a sliver layer needs L >= 2")
    hxy = 1.0 / n
    thick = np.full(L, 1.0 / L)
    s = L // 2
    if sliver:
        ts = hxy * sliver_ratio
        thick[:] = (1.0 - ts) / (L - 1)
        thick[s] = ts
    z_level = np.concatenate([[0.0], np.cumsum(thick)])
    z_level[-1] = 1.0
    n1 = n + 1
    kk, jj, ii = np.meshgrid(np.arange(L + 1), np.arange(n1), np.arange(n1), indexing="ij")
    ii = ii.ravel().astype(np.int64)
    jj = jj.ravel().astype(np.int64)
    kk = kk.ravel().astype(np.int64)
    n_nodes = ii.size
    per_level = n1 * n1
    Uxy = rng.uniform(-jitter, jitter, (L + 1, per_level, 2))
    if sliver:
        Uxy[s + 1] = Uxy[s]
    Uz = rng.uniform(-jitter, jitter, (L + 1, per_level))
    Uxy = Uxy.reshape(n_nodes, 2)
    Uz = Uz.reshape(n_nodes)
    boundary = (ii == 0) | (ii == n) | (jj == 0) | (jj == n) | (kk == 0) | (kk == L)
    Uxy[boundary] = 0.0
    Uz[boundary] = 0.0
    zscale = np.empty(L + 1)
    zscale[0] = zscale[L] = 0.0
    for k in range(1, L):
        zscale[k] = min(thick[k - 1], thick[k])
    nodes = np.empty((n_nodes, 3))
    nodes[:, 0] = ii * hxy + Uxy[:, 0] * hxy
    nodes[:, 1] = jj * hxy + Uxy[:, 1] * hxy
    nodes[:, 2] = z_level[kk] + Uz * zscale[kk]

    def nid(i, j, k):
        return i + n1 * (j + n1 * k)

    lay, cj, ci = np.meshgrid(np.arange(L), np.arange(n), np.arange(n), indexing="ij")
    ci = ci.ravel().astype(np.int64)
    cj = cj.ravel().astype(np.int64)
    lay = lay.ravel().astype(np.int64)
    n_col = ci.size
    conn = np.empty((n_col, 2, 6), dtype=np.int64)
    tris = (((0, 0), (1, 0), (1, 1)), ((0, 0), (1, 1), (0, 1)))
    for t, tri in enumerate(tris):
        for v, (di, dj) in enumerate(tri):
            conn[:, t, v] = nid(ci + di, cj + dj, lay)
            conn[:, t, v + 3] = nid(ci + di, cj + dj, lay + 1)
    conn = conn.reshape(n_col * 2, 6)
    return Mesh("prism6", _soa(nodes, conn), nodes, conn, boundary)


def tet_n_for(n_target: int) -> int:
    """Grid size N whose tet cube has about ``n_target`` elements."""
    return max(1, int(round((n_target / 6.0) ** (1.0 / 3.0))))


def prism_n_for(n_target: int) -> int:
    """Grid size n (= L) whose prism mesh has about ``n_target`` elements."""
    return max(1, int(round((n_target / 2.0) ** (1.0 / 3.0))))


# --------------------------------------------------------------------------
# Coefficient sets.
# --------------------------------------------------------------------------

N_SCALAR_SLOTS = 20
N_ELAST_SLOTS = 5
ALL_SCALAR_MASK = (1 << N_SCALAR_SLOTS) - 1
ALL_ELAST_MASK = (1 << N_ELAST_SLOTS) - 1
DIFF_SLOTS = (5, 6, 7, 9, 10, 11, 13, 14, 15)


def identity_diffusion_uniform(d0: float = 1.0) -> np.ndarray:
    """Twenty uniform slot values for the Poisson problem: c^{i;j} = identity,
    d^0 = ``d0``, all other coefficients zero."""
    u = np.zeros(N_SCALAR_SLOTS)
    u[5] = u[10] = u[15] = 1.0
    u[16] = d0
    return u


def cdr_per_element(n_elem: int, rng: np.random.Generator) -> np.ndarray:
    """All twenty convection-diffusion-reaction coefficients, constant per
    element, in the compact (20, n_elem) layout.

    Draw order: A ~ U[-1,1]^{3x3} giving c^{i;j} = A A^T + I/2 (symmetric
    positive definite); then c^{i;0}, c^{0;i}, d^i ~ U[-1,1]^3; then c^{0;0},
    d^0 ~ U[0,1]."""
    A = rng.uniform(-1.0, 1.0, (n_elem, 3, 3))
    cij = np.einsum("eik,ejk->eij", A, A) + 0.5 * np.eye(3)
    ci0 = rng.uniform(-1.0, 1.0, (n_elem, 3))
    c0i = rng.uniform(-1.0, 1.0, (n_elem, 3))
    di = rng.uniform(-1.0, 1.0, (n_elem, 3))
    c00 = rng.uniform(0.0, 1.0, n_elem)
    d0 = rng.uniform(0.0, 1.0, n_elem)
    out = np.empty((N_SCALAR_SLOTS, n_elem))
    out[0] = c00
    for i in range(3):
        out[1 + i] = c0i[:, i]
        out[4 * (i + 1)] = ci0[:, i]
        for j in range(3):
            out[4 * (i + 1) + 1 + j] = cij[:, i, j]
        out[17 + i] = di[:, i]
    out[16] = d0
    return out


def elasticity_per_element(n_elem: int, rng: np.random.Generator) -> np.ndarray:
    """Isotropic elasticity data per element, compact (5, n_elem) layout:
    E = exp(N(0, 0.5^2)), nu ~ U[0.2, 0.45], body force f ~ U[-1,1]^3."""
    E = np.exp(rng.normal(0.0, 0.5, n_elem))
    nu = rng.uniform(0.2, 0.45, n_elem)
    f = rng.uniform(-1.0, 1.0, (n_elem, 3))
    out = np.empty((N_ELAST_SLOTS, n_elem))
    out[0] = E
    out[1] = nu
    out[2:5] = f.T
    return out


N_VECTOR_SLOTS = 156
ALL_VECTOR_MASK = (1 << 20) - 1   # one bit per block of the 3-component problem


def vector_slot(a: int, b: int | None, alpha: int, beta: int | None = None) -> int:
    """Slot of c^{a;b}_{alpha beta} (b, beta given) or d^a_alpha (b None)."""
    if b is None:
        return 144 + 3 * a + alpha
    return (4 * a + b) * 9 + 3 * alpha + beta


def vector_block_rows(mask: int) -> int:
    """Rows of the compact coefficient array of a 3-component problem."""
    return sum((9 if k < 16 else 3) for k in range(20) if mask >> k & 1)


def vector_per_element(n_elem: int, rng: np.random.Generator) -> np.ndarray:
    """All 156 coefficients of the general 3-component problem, constant per
    element, (156, n_elem) in slot order.

    Draw order: B ~ U[-1,1]^{9x9} giving the diffusion tensor over the index
    pairs (i alpha), (j beta) as B B^T / 9 + I/2 (positive definite, so the
    operator is strongly elliptic); then c^{i;0}, c^{0;i} ~ U[-1,1]^{3x3x3},
    c^{0;0} ~ U[0,1]^{3x3}, d^i ~ U[-1,1]^{3x3}, d^0 ~ U[-1,1]^3."""
    B = rng.uniform(-1.0, 1.0, (n_elem, 9, 9))
    D = np.matmul(B, B.transpose(0, 2, 1)) / 9.0 + 0.5 * np.eye(9)   # [(3i+alpha), (3j+beta)]
    ci0 = rng.uniform(-1.0, 1.0, (n_elem, 3, 3, 3))   # [i, alpha, beta]
    c0i = rng.uniform(-1.0, 1.0, (n_elem, 3, 3, 3))
    c00 = rng.uniform(0.0, 1.0, (n_elem, 3, 3))
    di = rng.uniform(-1.0, 1.0, (n_elem, 3, 3))       # [i, alpha]
    d0 = rng.uniform(-1.0, 1.0, (n_elem, 3))
    out = np.zeros((N_VECTOR_SLOTS, n_elem))
    for al in range(3):
        for be in range(3):
            out[vector_slot(0, 0, al, be)] = c00[:, al, be]
            for i in range(3):
                out[vector_slot(i + 1, 0, al, be)] = ci0[:, i, al, be]
                out[vector_slot(0, i + 1, al, be)] = c0i[:, i, al, be]
                for j in range(3):
                    out[vector_slot(i + 1, j + 1, al, be)] = D[:, 3 * i + al, 3 * j + be]
        for i in range(3):
            out[vector_slot(i + 1, None, al)] = di[:, i, al]
        out[vector_slot(0, None, al)] = d0[:, al]
    return out


def vector_compact(full: np.ndarray, mask: int, n_q: int = 1) -> np.ndarray:
    """Keep the rows of the blocks present in ``mask`` (slot order); for
    per-point data ``full`` is (156 * n_q, n) with rows slot * n_q + q."""
    rows = []
    for k in range(20):
        if mask >> k & 1:
            base = k * 9 if k < 16 else 144 + 3 * (k - 16)
            for c in range(9 if k < 16 else 3):
                rows.extend((base + c) * n_q + q for q in range(n_q))
    return np.ascontiguousarray(full[rows])


def rhs_per_qp(n_elem: int, n_q: int, rng: np.random.Generator) -> np.ndarray:
    """A right-hand side d^0 ~ U[0,1] per quadrature point (the paper's
    "Poisson" input of one coefficient per point), compact (n_q, n_elem)."""
    return rng.uniform(0.0, 1.0, (n_q, n_elem))


# Sample points inside a prism at which smooth coefficient fields are
# evaluated: three interior triangle points (2/3,1/6), (1/6,2/3), (1/6,1/6) in
# the bottom-triangle barycentric frame, each at two heights (1 -+ 1/sqrt 3)/2
# of the way from the bottom face to the top face, point index 2 t + l. They
# are placed where the built-in 6-point prism rule puts its points, so the
# per-point data reads as "coefficient values at the quadrature points"; the
# exact locations do not affect any comparison because both the GPU path and
# the oracle consume the stored values.
_TRI_PTS = ((2.0 / 3.0, 1.0 / 6.0), (1.0 / 6.0, 2.0 / 3.0), (1.0 / 6.0, 1.0 / 6.0))
_HEIGHTS = ((1.0 - 1.0 / math.sqrt(3.0)) / 2.0, (1.0 + 1.0 / math.sqrt(3.0)) / 2.0)


def prism_sample_weights() -> np.ndarray:
    """(6, 6) convex weights: sample point p = sum_v W[p, v] * vertex_v."""
    W = np.zeros((6, 6))
    for t, (a, b) in enumerate(_TRI_PTS):
        bary = (1.0 - a - b, a, b)
        for l, hgt in enumerate(_HEIGHTS):
            p = 2 * t + l
            for v in range(3):
                W[p, v] = bary[v] * (1.0 - hgt)
                W[p, v + 3] = bary[v] * hgt
    return W


def smooth_cdr_per_qp(coords: np.ndarray, sample_w: np.ndarray, rng: np.random.Generator,
                      chunk: int = 1 << 20, dtype=np.float64) -> np.ndarray:
    """Twenty smooth coefficient fields sampled at n_q points per element.

    For each slot k: alpha_k ~ U[-1,1], beta_k ~ U[0,0.5], wave vector
    omega_k in {1,2,3}^3, phase theta_k ~ U[0, 2 pi); the field is
    alpha_k + beta_k sin(2 pi omega_k . x + theta_k). The diffusion block is
    then replaced by A A^T + I/2 with A read from slots 5-7, 9-11, 13-15 (so it
    is symmetric positive definite at every point), and c^{0;0}, d^0 are mapped
    to [0, 1] as 1/2 + 1/2 sin(...). Returns the compact per-point layout
    (20 * n_q, n_elem), row j * n_q + q."""
    n_q, n_vert = sample_w.shape
    n_elem = coords.shape[1]
    alpha = rng.uniform(-1.0, 1.0, N_SCALAR_SLOTS)
    beta = rng.uniform(0.0, 0.5, N_SCALAR_SLOTS)
    omega = rng.integers(1, 4, (N_SCALAR_SLOTS, 3))
    theta = rng.uniform(0.0, 2.0 * math.pi, N_SCALAR_SLOTS)
    out = np.empty((N_SCALAR_SLOTS * n_q, n_elem), dtype=dtype)
    X = coords.reshape(n_vert, 3, n_elem)
    for e0 in range(0, n_elem, chunk):
        e1 = min(n_elem, e0 + chunk)
        # sample points (n_q, 3, m)
        P = np.einsum("pv,vdm->pdm", sample_w, X[:, :, e0:e1])
        vals = np.empty((N_SCALAR_SLOTS, n_q, e1 - e0))
        for k in range(N_SCALAR_SLOTS):
            arg = 2.0 * math.pi * np.einsum("d,pdm->pm", omega[k].astype(np.float64), P) + theta[k]
            s = np.sin(arg)
            if k in (0, 16):
                vals[k] = 0.5 + 0.5 * s
            else:
                vals[k] = alpha[k] + beta[k] * s
        A = np.empty((3, 3, n_q, e1 - e0))
        for i in range(3):
            for j in range(3):
                A[i, j] = vals[4 * (i + 1) + 1 + j]
        for i in range(3):
            for j in range(3):
                cij = A[i, 0] * A[j, 0] + A[i, 1] * A[j, 1] + A[i, 2] * A[j, 2]
                if i == j:
                    cij = cij + 0.5
                vals[4 * (i + 1) + 1 + j] = cij
        out[:, e0:e1] = vals.reshape(N_SCALAR_SLOTS * n_q, e1 - e0)
    return out


# --------------------------------------------------------------------------
# The configurations the library is measured and tested on.
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    elem: str            # "tet4" | "prism6"
    kind: str            # "scalar" | "elasticity" | "vector"
    n_q: int
    coef_mode: str       # "uniform" | "element" | "qp"
    mask: int            # which slots are read from the coefficient array
    uniform: np.ndarray  # values of the remaining slots
    k_format: str        # "packed" | "full"
    mesh: Mesh
    coeffs: np.ndarray | None  # compact layout, float64

    @property
    def n_elem(self) -> int:
        return self.mesh.n_elem


def tet_poisson(N: int, seed: int = 1) -> Workload:
    """Scalar Poisson on the jittered tet cube: c^{i;j} = I, d^0 = 1 uniform,
    1-point rule, packed K (the headline workload; N = 8 gives 3,072
    elements, N = 119 gives 10,110,954)."""
    mesh = tet_cube(N, seed)
    return Workload("tet_poisson", "tet4", "scalar", 1, "uniform", 0,
                    identity_diffusion_uniform(1.0), "packed", mesh, None)


def tet_poisson_qp_rhs(N: int, seed: int = 1) -> Workload:
    """The paper's tetrahedral "Poisson" shape: Laplacian, d^0 given per
    quadrature point of the 4-point rule, full K (36 words per element)."""
    rng = np.random.default_rng(seed)
    mesh = tet_cube(N, rng)
    coeffs = rhs_per_qp(mesh.n_elem, 4, rng)
    return Workload("tet_poisson_qp", "tet4", "scalar", 4, "qp", 1 << 16,
                    identity_diffusion_uniform(0.0), "full", mesh, coeffs)


def tet_cdr(N: int, seed: int = 2) -> Workload:
    """Full convection-diffusion-reaction, coefficients per element, 4-point
    rule, full K."""
    rng = np.random.default_rng(seed)
    mesh = tet_cube(N, rng)
    coeffs = cdr_per_element(mesh.n_elem, rng)
    return Workload("tet_cdr", "tet4", "scalar", 4, "element", ALL_SCALAR_MASK,
                    np.zeros(N_SCALAR_SLOTS), "full", mesh, coeffs)


def prism_cdr_qp(n: int, L: int, seed: int = 3, sliver: bool = True) -> Workload:
    """Prisms with all twenty coefficients given per quadrature point as smooth
    fields, 6-point rule, full K."""
    rng = np.random.default_rng(seed)
    mesh = prism_layers(n, L, rng, sliver=sliver)
    coeffs = smooth_cdr_per_qp(mesh.coords, prism_sample_weights(), rng)
    return Workload("prism_cdr_qp", "prism6", "scalar", 6, "qp", ALL_SCALAR_MASK,
                    np.zeros(N_SCALAR_SLOTS), "full", mesh, coeffs)


def prism_cdr_element(n: int, L: int, seed: int = 3, sliver: bool = True) -> Workload:
    """Prisms with the twenty coefficients constant per element."""
    rng = np.random.default_rng(seed)
    mesh = prism_layers(n, L, rng, sliver=sliver)
    coeffs = cdr_per_element(mesh.n_elem, rng)
    return Workload("prism_cdr", "prism6", "scalar", 6, "element", ALL_SCALAR_MASK,
                    np.zeros(N_SCALAR_SLOTS), "full", mesh, coeffs)


def tet_elasticity(N: int, seed: int = 4) -> Workload:
    """3-component isotropic elasticity on tets, per-element (E, nu, f),
    1-point rule, packed K."""
    rng = np.random.default_rng(seed)
    mesh = tet_cube(N, rng)
    coeffs = elasticity_per_element(mesh.n_elem, rng)
    return Workload("tet_elasticity", "tet4", "elasticity", 1, "element", ALL_ELAST_MASK,
                    np.zeros(N_ELAST_SLOTS), "packed", mesh, coeffs)


def prism_elasticity(n: int, L: int, seed: int = 4, sliver: bool = True) -> Workload:
    """3-component isotropic elasticity on prisms, per-element (E, nu, f),
    6-point rule, packed K."""
    rng = np.random.default_rng(seed)
    mesh = prism_layers(n, L, rng, sliver=sliver)
    coeffs = elasticity_per_element(mesh.n_elem, rng)
    return Workload("prism_elasticity", "prism6", "elasticity", 6, "element", ALL_ELAST_MASK,
                    np.zeros(N_ELAST_SLOTS), "packed", mesh, coeffs)


def prism_poisson_qp_rhs(n: int, L: int, seed: int = 3, sliver: bool = True) -> Workload:
    """The paper's prismatic "Poisson" shape: Laplacian, d^0 given per point
    of the 6-point rule, full K (66 words per element)."""
    rng = np.random.default_rng(seed)
    mesh = prism_layers(n, L, rng, sliver=sliver)
    coeffs = rhs_per_qp(mesh.n_elem, 6, rng)
    return Workload("prism_poisson_qp", "prism6", "scalar", 6, "qp", 1 << 16,
                    identity_diffusion_uniform(0.0), "full", mesh, coeffs)


# --------------------------------------------------------------------------
# Coefficient functions: parameters instead of values.
# --------------------------------------------------------------------------
def tet_vector(N: int, seed: int = 6) -> Workload:
    """General 3-component convection-diffusion-reaction on tets: all 156
    coefficients per element, 4-point rule, full 12x12 K."""
    rng = np.random.default_rng(seed)
    mesh = tet_cube(N, rng)
    coeffs = vector_per_element(mesh.n_elem, rng)
    return Workload("tet_vector", "tet4", "vector", 4, "element", ALL_VECTOR_MASK,
                    np.zeros(N_SCALAR_SLOTS), "full", mesh, coeffs)


def prism_vector(n: int, L: int, seed: int = 7, sliver: bool = True) -> Workload:
    """General 3-component problem on prisms, 156 coefficients per element,
    6-point rule, full 18x18 K."""
    rng = np.random.default_rng(seed)
    mesh = prism_layers(n, L, rng, sliver=sliver)
    coeffs = vector_per_element(mesh.n_elem, rng)
    return Workload("prism_vector", "prism6", "vector", 6, "element", ALL_VECTOR_MASK,
                    np.zeros(N_SCALAR_SLOTS), "full", mesh, coeffs)


def reordered(wl: Workload, order: str = "morton") -> Workload:
    """A workload on the Z-order renumbered mesh, per-element or per-point
    coefficients permuted with the elements."""
    if order != "morton":
        return wl
    mesh, perm = morton_order(wl.mesh)
    coeffs = wl.coeffs
    if coeffs is not None and wl.coef_mode in ("element", "qp"):
        coeffs = np.ascontiguousarray(coeffs[:, perm])
    return Workload(wl.name, wl.elem, wl.kind, wl.n_q, wl.coef_mode, wl.mask, wl.uniform,
                    wl.k_format, mesh, coeffs)


N_FN_PARAMS = 122


def smooth_cdr_params(rng: np.random.Generator, spd_shift: float = 0.5) -> np.ndarray:
    """Parameters of the smooth coefficient fields of smooth_cdr_per_qp, in the
    same draw order, for the function mode: row k of the (122,) table holds
    (alpha_k, beta_k, omega_k, theta_k) at [6k .. 6k+5]; slots 0 and 16 get
    alpha = beta = 1/2 (the [0, 1] mapping); [120] is the shift of the SPD
    diffusion transform and [121] = 1 enables it."""
    alpha = rng.uniform(-1.0, 1.0, N_SCALAR_SLOTS)
    beta = rng.uniform(0.0, 0.5, N_SCALAR_SLOTS)
    omega = rng.integers(1, 4, (N_SCALAR_SLOTS, 3))
    theta = rng.uniform(0.0, 2.0 * math.pi, N_SCALAR_SLOTS)
    p = np.zeros(N_FN_PARAMS)
    for k in range(N_SCALAR_SLOTS):
        a, b = (0.5, 0.5) if k in (0, 16) else (alpha[k], beta[k])
        p[6 * k: 6 * k + 6] = (a, b, omega[k, 0], omega[k, 1], omega[k, 2], theta[k])
    p[120] = spd_shift
    p[121] = 1.0
    return p


def prism_cdr_fn(n: int, L: int, seed: int = 3, sliver: bool = True) -> Workload:
    """Prisms with all twenty coefficients computed at the points from the
    smooth-field parameters (the per-point workload's fields, evaluated in the
    kernel instead of read from memory)."""
    rng = np.random.default_rng(seed)
    mesh = prism_layers(n, L, rng, sliver=sliver)
    return Workload("prism_cdr_fn", "prism6", "scalar", 6, "function", ALL_SCALAR_MASK,
                    np.zeros(N_SCALAR_SLOTS), "full", mesh, smooth_cdr_params(rng))


def tet_cdr_fn(N: int, seed: int = 2) -> Workload:
    """Tets with the twenty coefficients as smooth functions of position,
    4-point rule, full K."""
    rng = np.random.default_rng(seed)
    mesh = tet_cube(N, rng)
    return Workload("tet_cdr_fn", "tet4", "scalar", 4, "function", ALL_SCALAR_MASK,
                    np.zeros(N_SCALAR_SLOTS), "full", mesh, smooth_cdr_params(rng))
