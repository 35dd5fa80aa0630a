"""P1 finite elements on the unit square / cube (oracle; test infrastructure only).

Follows the discretization of the paper's Sec. 3: H^1-conforming continuous P1
(Lagrange) elements on Omega = (0,1)^d, and a P1 trace space on Gamma whose degrees
of freedom are point evaluations, so the discrete trace T_h is nodal injection.

Reading of the geometry (the paper's eq. (riesz) names V = H^1_0 with Gamma on the
boundary, which cannot hold literally): Gamma is the top facet {x_d = 1}; homogeneous
Dirichlet conditions hold on the rest of the boundary, and the nodes on the closure
of Gamma's boundary are Dirichlet too.  The interface Laplacian therefore carries
homogeneous Dirichlet conditions at the boundary of Gamma.

Meshes
  2D: nodes (i h, j h), i, j = 0..n, h = 1/n.  Each cell is split along the diagonal
      from (i, j) to (i+1, j+1).
  3D: nodes (i h, j h, k h).  Each cube cell is split into the six Kuhn
      tetrahedra  v, v+e_a, v+e_a+e_b, v+(1,1,1)  over the permutations (a, b, c).

Free-dof order (Gamma last)
  2D: index (j-1)(n-1) + (i-1),  j = 1..n, i = 1..n-1;  Gamma is j = n.
  3D: index ((k-1)(n-1) + (j-1))(n-1) + (i-1),  i, j = 1..n-1, k = 1..n;  Gamma is k = n.

Assembly is done element by element from the generic P1 formulas
  stiffness  a_T(i, j) = |T| grad(lambda_i) . grad(lambda_j)
  mass       m_T(i, j) = |T| (1 + delta_ij) / ((d+1)(d+2))
with no stencil assumed anywhere.

Parity: pinned by tests against the closed-form 1D eigenpairs, the Dirichlet
Laplacian row sums, the Galerkin identity for nested meshes and brute-force
consistency with the separable sine-transform solver.
"""
import itertools

import numpy as np
import scipy.sparse as sp


# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------

def mesh_2d(n):
    """Nodes (N, 2) and triangles (T, 3) of the uniform right-triangle mesh."""
    h = 1.0 / n
    I, J = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    nodes = np.stack([I.ravel() * h, J.ravel() * h], axis=1)

    def nid(i, j):
        return j * (n + 1) + i

    tris = []
    for j in range(n):
        for i in range(n):
            # split along the diagonal (i, j) -> (i+1, j+1)
            tris.append((nid(i, j), nid(i + 1, j), nid(i + 1, j + 1)))
            tris.append((nid(i, j), nid(i + 1, j + 1), nid(i, j + 1)))
    return nodes, np.array(tris, dtype=np.int64)


def mesh_3d(n):
    """Nodes (N, 3) and Kuhn tetrahedra (T, 4) of the uniform cube mesh."""
    h = 1.0 / n
    idx = np.arange(n + 1)
    K, J, I = np.meshgrid(idx, idx, idx, indexing="ij")
    nodes = np.stack([I.ravel() * h, J.ravel() * h, K.ravel() * h], axis=1)

    def nid(i, j, k):
        return (k * (n + 1) + j) * (n + 1) + i

    unit = [np.array(e) for e in ((1, 0, 0), (0, 1, 0), (0, 0, 1))]
    tets = []
    for k in range(n):
        for j in range(n):
            for i in range(n):
                v = np.array((i, j, k))
                for perm in itertools.permutations(range(3)):
                    a = v + unit[perm[0]]
                    b = a + unit[perm[1]]
                    c = v + 1
                    tets.append((nid(*v), nid(*a), nid(*b), nid(*c)))
    return nodes, np.array(tets, dtype=np.int64)


# ----------------------------------------------------------------------------
# generic P1 element matrices and assembly
# ----------------------------------------------------------------------------

def p1_element_matrices(coords):
    """Element stiffness and mass for one simplex.

    coords: (d+1, d) vertex coordinates.  Returns (A_T, M_T), each (d+1, d+1).
    Barycentric gradients come from x = x0 + B xi, grad xi_k = row k of B^{-1},
    grad lambda_0 = -sum_k grad xi_k.
    """
    d = coords.shape[1]
    B = (coords[1:] - coords[0]).T                      # (d, d)
    Binv = np.linalg.inv(B)
    grads = np.vstack([-Binv.sum(axis=0), Binv])        # (d+1, d)
    vol = abs(np.linalg.det(B)) / np.prod(np.arange(1, d + 1))
    A_T = vol * grads @ grads.T
    M_T = vol * (np.ones((d + 1, d + 1)) + np.eye(d + 1)) / ((d + 1) * (d + 2))
    return A_T, M_T


def assemble(nodes, cells):
    """Global stiffness and mass (all nodes), summed element by element."""
    nn = nodes.shape[0]
    k = cells.shape[1]
    rows, cols, av, mv = [], [], [], []
    for cell in cells:
        A_T, M_T = p1_element_matrices(nodes[cell])
        r = np.repeat(cell, k)
        c = np.tile(cell, k)
        rows.append(r)
        cols.append(c)
        av.append(A_T.ravel())
        mv.append(M_T.ravel())
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    A = sp.coo_matrix((np.concatenate(av), (rows, cols)), shape=(nn, nn)).tocsr()
    M = sp.coo_matrix((np.concatenate(mv), (rows, cols)), shape=(nn, nn)).tocsr()
    A.sum_duplicates()
    M.sum_duplicates()
    return A, M


# ----------------------------------------------------------------------------
# free dofs, interface, problem container
# ----------------------------------------------------------------------------

def free_dofs(dim, n):
    """Global node numbers of the free dofs, in the oracle order (Gamma last)."""
    if dim == 2:
        out = [j * (n + 1) + i for j in range(1, n + 1) for i in range(1, n)]
    elif dim == 3:
        out = [(k * (n + 1) + j) * (n + 1) + i
               for k in range(1, n + 1) for j in range(1, n) for i in range(1, n)]
    else:
        raise ValueError("dim must be 2 or 3")
    return np.array(out, dtype=np.int64)


def sizes(dim, n):
    """(N, N_I, N_Gamma) for the free dofs."""
    if dim == 2:
        return n * (n - 1), (n - 1) ** 2, n - 1
    return n * (n - 1) ** 2, (n - 1) ** 3, (n - 1) ** 2


def interface_mesh(dim, n):
    """Gamma's own P1 mesh: nodes in Gamma coordinates and cells.

    2D: segments of the line y = 1.  3D: the faces of the Kuhn tetrahedra that lie in
    z = 1 (found from the tetrahedra, so the face diagonal follows the volume mesh).
    """
    if dim == 2:
        h = 1.0 / n
        nodes = (np.arange(n + 1) * h)[:, None]
        cells = np.array([(i, i + 1) for i in range(n)], dtype=np.int64)
        return nodes, cells
    nodes3, tets = mesh_3d(n)
    top = np.isclose(nodes3[:, 2], 1.0)
    faces = set()
    for t in tets:
        on = [v for v in t if top[v]]
        if len(on) == 3:
            faces.add(tuple(sorted(on)))
    # renumber top nodes as j*(n+1)+i
    faces = np.array(sorted(faces), dtype=np.int64)
    glob_to_face = {}
    for g in np.nonzero(top)[0]:
        i = int(round(nodes3[g, 0] * n))
        j = int(round(nodes3[g, 1] * n))
        glob_to_face[g] = j * (n + 1) + i
    cells = np.vectorize(glob_to_face.get)(faces)
    h = 1.0 / n
    I, J = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    fnodes = np.stack([I.ravel() * h, J.ravel() * h], axis=1)
    return fnodes, cells


def interface_free(dim, n):
    """Free interface nodes in Gamma numbering, in the order of the last N_Gamma dofs."""
    if dim == 2:
        return np.arange(1, n, dtype=np.int64)
    return np.array([j * (n + 1) + i for j in range(1, n) for i in range(1, n)], dtype=np.int64)


class Problem:
    """Assembled FP64 matrices of one (dim, n) instance.

    Attributes
      A      free-dof stiffness of -Delta (K not included), sparse CSR (N, N)
      A_G    interface stiffness (L_h), dense (N_G, N_G)
      M_G    interface mass (M_h), dense (N_G, N_G)
      N, NI, NG   sizes
    """

    def __init__(self, dim, n):
        if n < 2:
            raise ValueError("n must be >= 2")
        self.dim, self.n = dim, n
        nodes, cells = mesh_2d(n) if dim == 2 else mesh_3d(n)
        A_all, _ = assemble(nodes, cells)
        fd = free_dofs(dim, n)
        self.A = A_all[fd][:, fd].tocsr()
        self.N, self.NI, self.NG = sizes(dim, n)
        gn, gc = interface_mesh(dim, n)
        AG_all, MG_all = assemble(gn, gc)
        gf = interface_free(dim, n)
        self.A_G = AG_all[gf][:, gf].toarray()
        self.M_G = MG_all[gf][:, gf].toarray()

    # block views of the stiffness (interior I first, Gamma last)
    def blocks(self):
        NI = self.NI
        A = self.A
        return (A[:NI, :NI].tocsc(), A[:NI, NI:].tocsc(),
                A[NI:, :NI].tocsc(), A[NI:, NI:].toarray())
