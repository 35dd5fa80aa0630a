// Host set-up of the H(div) problem (Sec. 3, remark on H(div)-elliptic problems, eq. (graddiv)):
// lowest-order BDM fields on the diagonal-split mesh, the matrices of every multigrid level, the
// transfers between nested levels, the vertex-patch tables of the smoother and the blocks of the
// trace operator L on the boundary loop.
//
// BDM1 basis.  On a triangle with edge e = (a, b) (a, b local vertices, n_e the edge's normal),
// the field of the dof "u.n_e at a" is lambda_a w with the constant field
// w = curl lambda_b / (curl lambda_b . n_e), curl phi = (d_y phi, -d_x phi): curl lambda_b is
// parallel to the edge opposite b, so the field's normal component vanishes on the two other
// edges, and on e it is lambda_a.  Mass entries are (w . w') |T| (1 + [a = a']) / 12 and the
// divergence is grad lambda_a . w.
//
// Geometry is computed from integer vertex offsets (then scaled by h), so congruent triangles
// give bit-identical element matrices and congruent vertex patches bit-identical patch matrices.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ell_host.h"
#include "hdiv_internal.h"

namespace fdd {

namespace {

struct Edge {
  int pi, pj, qi, qj;   // first and second endpoint (grid coordinates)
  double nx, ny;        // normal
};

int edges_interior(int n) { return 3 * n * n - 2 * n; }

// Edge index and endpoints in the documented order (interior horizontal, vertical, diagonal,
// then the boundary loop).
Edge edge_at(int n, int e) {
  const int nh = n * (n - 1), nv = (n - 1) * n, nd = n * n;
  const double s = 1.0 / std::sqrt(2.0);
  if (e < nh) {
    const int j = e / n + 1, i = e % n;
    return {i, j, i + 1, j, 0.0, 1.0};
  }
  e -= nh;
  if (e < nv) {
    const int j = e / (n - 1), i = e % (n - 1) + 1;
    return {i, j, i, j + 1, 1.0, 0.0};
  }
  e -= nv;
  if (e < nd) {
    const int j = e / n, i = e % n;
    return {i, j, i + 1, j + 1, s, -s};
  }
  e -= nd;
  const int side = e / n, k = e % n;
  switch (side) {
    case 0: return {k, 0, k + 1, 0, 0.0, -1.0};
    case 1: return {n, k, n, k + 1, 1.0, 0.0};
    case 2: return {n - k, n, n - k - 1, n, 0.0, 1.0};
    default: return {0, n - k, 0, n - k - 1, -1.0, 0.0};
  }
}

// Index of the edge between grid vertices (ai, aj) and (bi, bj) (any order).
int edge_between(int n, int ai, int aj, int bi, int bj) {
  const int ni = edges_interior(n);
  if (aj == bj) {                     // horizontal
    const int i = std::min(ai, bi), j = aj;
    if (j == 0) return ni + i;
    if (j == n) return ni + 2 * n + (n - 1 - i);
    return (j - 1) * n + i;
  }
  if (ai == bi) {                     // vertical
    const int i = ai, j = std::min(aj, bj);
    if (i == 0) return ni + 3 * n + (n - 1 - j);
    if (i == n) return ni + n + j;
    return n * (n - 1) + j * (n - 1) + (i - 1);
  }
  const int i = std::min(ai, bi), j = std::min(aj, bj);  // diagonal
  return 2 * n * (n - 1) + j * n + i;
}

// The six local fields of one triangle.
struct Local {
  int dof[6];
  int vert[6];          // local vertex a of the field lambda_a w
  double w[6][2];
  double div[6];
  double area;
  double grad[3][2];
  int vi[3], vj[3];     // grid coordinates of the vertices
};

// Triangle t of cell (ci, cj): t = 0 lower (v, v + (1,0), v + (1,1)), t = 1 upper
// (v, v + (1,1), v + (0,1)).
Local local_fields(int n, int ci, int cj, int t) {
  Local L{};
  static const int off[2][3][2] = {{{0, 0}, {1, 0}, {1, 1}}, {{0, 0}, {1, 1}, {0, 1}}};
  const double h = 1.0 / n;
  for (int a = 0; a < 3; ++a) {
    L.vi[a] = ci + off[t][a][0];
    L.vj[a] = cj + off[t][a][1];
  }
  // barycentric gradients from the offsets: B = [x1 - x0, x2 - x0] (columns), grad xi = rows of B^-1
  const double b00 = (off[t][1][0] - off[t][0][0]) * h, b10 = (off[t][1][1] - off[t][0][1]) * h;
  const double b01 = (off[t][2][0] - off[t][0][0]) * h, b11 = (off[t][2][1] - off[t][0][1]) * h;
  const double det = b00 * b11 - b01 * b10;
  // B^-1 = [[b11, -b01], [-b10, b00]] / det; grad lambda_1 = row 0, grad lambda_2 = row 1
  L.grad[1][0] = b11 / det;
  L.grad[1][1] = -b01 / det;
  L.grad[2][0] = -b10 / det;
  L.grad[2][1] = b00 / det;
  L.grad[0][0] = -(L.grad[1][0] + L.grad[2][0]);
  L.grad[0][1] = -(L.grad[1][1] + L.grad[2][1]);
  L.area = std::fabs(det) / 2.0;
  int k = 0;
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b) {
      if (a == b) continue;
      const int e = edge_between(n, L.vi[a], L.vj[a], L.vi[b], L.vj[b]);
      const Edge E = edge_at(n, e);
      const bool first = (E.pi == L.vi[a] && E.pj == L.vj[a]);
      const double cx = L.grad[b][1], cy = -L.grad[b][0];  // curl lambda_b
      const double cn = cx * E.nx + cy * E.ny;
      L.dof[k] = 2 * e + (first ? 0 : 1);
      L.vert[k] = a;
      L.w[k][0] = cx / cn;
      L.w[k][1] = cy / cn;
      L.div[k] = L.grad[a][0] * L.w[k][0] + L.grad[a][1] * L.w[k][1];
      ++k;
    }
  }
  return L;
}

// Assembles K(mass + div-div) of level n: rows/cols below n0 only (interior == true: A^00), or
// every dof plus gamma times the boundary mass of (u.nu)(v.nu) (the whole operator).
void assemble(int n, double K, double gamma, bool interior, RowBuilder* rb) {
  const int n0 = 2 * edges_interior(n);
  for (int cj = 0; cj < n; ++cj)
    for (int ci = 0; ci < n; ++ci)
      for (int t = 0; t < 2; ++t) {
        const Local L = local_fields(n, ci, cj, t);
        for (int a = 0; a < 6; ++a) {
          if (interior && L.dof[a] >= n0) continue;
          for (int b = 0; b < 6; ++b) {
            if (interior && L.dof[b] >= n0) continue;
            const double same = (L.vert[a] == L.vert[b]) ? 2.0 : 1.0;
            const double m = (L.w[a][0] * L.w[b][0] + L.w[a][1] * L.w[b][1]) * L.area * same / 12.0;
            const double d = L.area * L.div[a] * L.div[b];
            rb->add(L.dof[a], L.dof[b], K * (m + d));
          }
        }
      }
  if (!interior) {
    // gamma int (u.nu)(v.nu) on each boundary segment: (h/6)[[2, 1], [1, 2]] on its two dofs
    const double h = 1.0 / n;
    for (int k = 0; k < 4 * n; ++k) {
      const int a = n0 + 2 * k, b = a + 1;
      rb->add(a, a, gamma * 2.0 * h / 6.0);
      rb->add(b, b, gamma * 2.0 * h / 6.0);
      rb->add(a, b, gamma * h / 6.0);
      rb->add(b, a, gamma * h / 6.0);
    }
  }
}

// Prolongation from level nc = n / 2 to level n on the interior dofs: the fine dof "u.n_e at p"
// of a coarse field is its value at p (in the coarse triangle holding the fine edge) times n_e.
void build_prolongation(int n, HdLevel* fine) {
  const int nc = n / 2, n0 = 2 * edges_interior(n), n0c = 2 * edges_interior(nc);
  const double h = 1.0 / n;
  RowBuilder rb(n0, 6);
  for (int e = 0; e < n0 / 2; ++e) {
    const Edge E = edge_at(n, e);
    // midpoint in coarse cells: (p + q) / 4
    const double mx = (E.pi + E.qi) / 4.0, my = (E.pj + E.qj) / 4.0;
    const int ci = std::min((int)std::floor(mx), nc - 1), cj = std::min((int)std::floor(my), nc - 1);
    const double lx = mx - ci, ly = my - cj;
    const int t = (lx >= ly) ? 0 : 1;
    const Local C = local_fields(nc, ci, cj, t);
    const double hc = 1.0 / nc;
    const double x0 = C.vi[0] * hc, y0 = C.vj[0] * hc;
    for (int end = 0; end < 2; ++end) {
      const double px = (end ? E.qi : E.pi) * h, py = (end ? E.qj : E.pj) * h;
      // barycentric coordinates: lambda_a = 1/3-free form via the gradients
      double lam[3];
      lam[1] = C.grad[1][0] * (px - x0) + C.grad[1][1] * (py - y0);
      lam[2] = C.grad[2][0] * (px - x0) + C.grad[2][1] * (py - y0);
      lam[0] = 1.0 - lam[1] - lam[2];
      for (int a = 0; a < 6; ++a) {
        if (C.dof[a] >= n0c) continue;
        const double v = lam[C.vert[a]] * (C.w[a][0] * E.nx + C.w[a][1] * E.ny);
        if (std::fabs(v) > 1e-14) rb.add(2 * e + end, C.dof[a], v);
      }
    }
  }
  rb.to_ell(&fine->P, n0c);
  ell_transpose(fine->P, n0c, &fine->R);
}

// Vertex patches: the interior dofs on the edges incident to each vertex, ascending; patch
// matrices deduplicated into types (congruent patches are bit-identical).
const char* build_patches(HdLevel* L) {
  const int n = L->n, n0 = L->n0;
  static const int nb[6][2] = {{-1, 0}, {1, 0}, {0, -1}, {0, 1}, {-1, -1}, {1, 1}};
  return build_patch_tables(L, (n + 1) * (n + 1), kHdPatch, [&](int v, int* dofs) {
    const int i = v % (n + 1), j = v / (n + 1);
    int m = 0;
    for (int k = 0; k < 6; ++k) {
      const int bi = i + nb[k][0], bj = j + nb[k][1];
      if (bi < 0 || bi > n || bj < 0 || bj > n) continue;
      const int e = edge_between(n, i, j, bi, bj);
      if (2 * e >= n0) continue;
      dofs[m++] = 2 * e;
      dofs[m++] = 2 * e + 1;
    }
    return m;
  });
}

// Blocks of the trace operator on the loop (segment k holds u at its start and at its end):
// L = sum_e int (u'v' + uv) - sum_vertices ({u'}[v] + {v'}[u]) + (sigma / h) sum [u][v],
// [u] = u(end of the segment before the vertex) - u(start of the one after), {u'} the mean
// of the two segments' derivatives (u_end - u_start) / h.  Row segment k: `own` on itself,
// `prev` on segment k - 1, prev^T on segment k + 1; `mass` is M_Q's block.
constexpr double kSigma = 4.0;
void loop_blocks(int n, double own[4], double prev[4], double mass[4]) {
  const double h = 1.0 / n;
  mass[0] = mass[3] = 2.0 * h / 6.0;
  mass[1] = mass[2] = h / 6.0;
  // segment-local stiffness + mass
  own[0] = own[3] = 1.0 / h + mass[0];
  own[1] = own[2] = -1.0 / h + mass[1];
  // a vertex couples the segment before it (as "a": jump coefficient +1 on its end value,
  // derivative mean (-1/2h, 1/2h)) with the one after it (as "b": jump -1 on its start value,
  // derivative mean (-1/2h, 1/2h)).  Form: -(d_r j_c + j_r d_c) + (sigma/h) j_r j_c.
  const double ja[2] = {0.0, 1.0}, jb[2] = {-1.0, 0.0};
  const double da[2] = {-0.5 / h, 0.5 / h}, db[2] = {-0.5 / h, 0.5 / h};
  auto vert = [&](const double* dr, const double* jr, const double* dc, const double* jc, int r,
                  int c) { return -(dr[r] * jc[c] + jr[r] * dc[c]) + (kSigma / h) * jr[r] * jc[c]; };
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) {
      // segment k is "b" at its start vertex and "a" at its end vertex
      own[r * 2 + c] += vert(db, jb, db, jb, r, c) + vert(da, ja, da, ja, r, c);
      // row k (as b at vertex k), column k - 1 (as a)
      prev[r * 2 + c] = vert(db, jb, da, ja, r, c);
    }
}

}  // namespace

const char* hdiv_build(ProblemHdiv* Q, int n, double K, double gamma) {
  Q->n = n;
  Q->K = K;
  Q->gamma = gamma;
  Q->N0 = 2 * edges_interior(n);
  Q->NG = 8 * n;
  Q->N = Q->N0 + Q->NG;
  int nl = 0;
  for (int m = n; m >= std::min(n, kHdCoarseN); m /= 2) {
    if (nl == kHdMaxLevels) return "too many levels";
    HdLevel& L = Q->lev[nl++];
    L.n = m;
    L.n0 = 2 * edges_interior(m);
    RowBuilder rb(L.n0, 10);
    assemble(m, K, 0.0, true, &rb);
    if (rb.overflow) return "assembly: more couplings per row than the mesh allows";
    rb.to_ell(&L.A, L.n0);
    if (const char* err = build_patches(&L)) return err;
  }
  Q->nlev = nl;
  for (int l = 0; l + 1 < nl; ++l) build_prolongation(Q->lev[l].n, &Q->lev[l]);
  // coarsest level: dense inverse
  {
    const HdLevel& C = Q->lev[nl - 1];
    std::vector<double> A((size_t)C.n0 * C.n0);
    for (int i = 0; i < C.n0; ++i)
      for (int j = 0; j < C.n0; ++j) A[(size_t)i * C.n0 + j] = ell_entry(C.A, i, j);
    if (!spd_inverse(A, C.n0)) return "the coarsest matrix is not positive definite";
    Q->cinv = A;
  }
  // the whole operator and its blocks
  {
    RowBuilder rb(Q->N, 10);
    assemble(n, K, gamma, false, &rb);
    if (rb.overflow) return "assembly: more couplings per row than the mesh allows";
    rb.to_ell(&Q->Afull, Q->N);
    const int N0 = Q->N0, NG = Q->NG;
    RowBuilder r0g(N0, 10), rg0(NG, 10), rgg(NG, 10);
    for (int i = 0; i < Q->N; ++i)
      for (int k = 0; k < rb.cnt[i]; ++k) {
        const int j = rb.col[(size_t)i * rb.cap + k];
        const double v = rb.val[(size_t)i * rb.cap + k];
        if (i < N0 && j >= N0) r0g.add(i, j - N0, v);
        else if (i >= N0 && j < N0) rg0.add(i - N0, j, v);
        else if (i >= N0) rgg.add(i - N0, j - N0, v);
      }
    r0g.to_ell(&Q->A0G, NG);
    rg0.to_ell(&Q->AG0, N0);
    rgg.to_ell(&Q->AGG, NG);
  }
  loop_blocks(n, Q->blk.own, Q->blk.prev, Q->blk.mass);
  return nullptr;
}

std::vector<double> hdiv_loop_eigs(const ProblemHdiv* Q) {
  // for theta = 2 pi q / (4n): det(S(theta) - lam M) = 0 with the Hermitian symbol
  // S = own + prev e^{-i theta} + prev^T e^{i theta}
  const int m = 4 * Q->n;
  const double* own = Q->blk.own;
  const double* P = Q->blk.prev;
  const double* M = Q->blk.mass;
  std::vector<double> out;
  out.reserve(2 * (size_t)m);
  for (int q = 0; q < m; ++q) {
    const double th = 2.0 * M_PI * q / m, c = std::cos(th), s = std::sin(th);
    // entries: S_00, S_11 real; S_01 = own_01 + P_01 e^{-i th} + P_10 e^{i th}
    const double a = own[0] + 2.0 * P[0] * c;
    const double d = own[3] + 2.0 * P[3] * c;
    const double br = own[1] + (P[1] + P[2]) * c, bi = (P[2] - P[1]) * s;
    const double m11 = M[0], m22 = M[3], m12 = M[1];
    // (m11 m22 - m12^2) lam^2 - (a m22 + d m11 - 2 m12 br) lam + (a d - |b|^2) = 0
    const double A2 = m11 * m22 - m12 * m12;
    const double A1 = -(a * m22 + d * m11 - 2.0 * m12 * br);
    const double A0 = a * d - (br * br + bi * bi);
    const double disc = std::sqrt(std::max(A1 * A1 - 4.0 * A2 * A0, 0.0));
    // stable roots
    const double qq = -0.5 * (A1 + (A1 >= 0 ? disc : -disc));
    out.push_back(qq / A2);
    out.push_back(A0 / qq);
  }
  std::sort(out.begin(), out.end());
  return out;
}

size_t hdiv_plan(ProblemHdiv* Q, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = (off + 255) / 256 * 256;
    char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  auto mat = [&](HdMat& M) {
    // relative form: the per-type offsets replace the per-row columns on the device
    M.dcol = M.toff.empty() ? (int*)take(M.col.size() * sizeof(int)) : nullptr;
    M.dtoff = M.toff.empty() ? nullptr : (int*)take(M.toff.size() * sizeof(int));
    M.drtype = (int*)take(M.rtype.size() * sizeof(int));
    M.dtval = (double*)take(M.tval.size() * sizeof(double));
  };
  for (int l = 0; l < Q->nlev; ++l) {
    HdLevel& L = Q->lev[l];
    mat(L.A);
    if (l + 1 < Q->nlev) {
      mat(L.P);
      mat(L.R);
    }
    L.dpatch = (int*)take(L.patch.size() * sizeof(int));
    L.dptype = (int*)take(L.ptype.size() * sizeof(int));
    L.dslot = (int*)take(L.slot.size() * sizeof(int));
    L.dpinv = (double*)take(L.pinv.size() * sizeof(double));
    L.x = (double*)take((size_t)L.n0 * 8);
    L.b = (double*)take((size_t)L.n0 * 8);
    L.r = (double*)take((size_t)L.n0 * 8);
    L.Y = (double*)take((size_t)L.nvert * L.pw * 8);
  }
  Q->dcinv = (double*)take(Q->cinv.size() * 8);
  mat(Q->A0G);
  mat(Q->AG0);
  mat(Q->AGG);
  mat(Q->Afull);
  const size_t n0 = (size_t)Q->N0 * 8, ng = (size_t)Q->NG * 8;
  Q->u = (double*)take(n0);
  Q->r = (double*)take(n0);
  Q->z = (double*)take(n0);
  Q->p = (double*)take(2 * n0);
  Q->q = (double*)take(n0);
  Q->f = (double*)take(n0);
  Q->t0 = (double*)take(n0);
  Q->xG = (double*)take(ng);
  Q->rG = (double*)take(ng);
  Q->zG = (double*)take(ng);
  Q->pG = (double*)take(ng);
  Q->yG = (double*)take(ng);
  Q->tG = (double*)take(ng);
  Q->partials = (double*)take(2 * kHdPartials * 8);
  Q->scratch = (double*)take((size_t)(kMaxPoles + 2) * ng);
  Q->st = (HdState*)take(sizeof(HdState));
  return (off + 255) / 256 * 256;
}

}  // namespace fdd
