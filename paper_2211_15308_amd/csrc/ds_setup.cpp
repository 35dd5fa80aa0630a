// Host set-up of the Darcy-Stokes problem (Sec. 4, eq. (darcy_stokes)): Taylor-Hood P2-P1
// matrices of the Stokes part, the P1 Darcy stiffness, the interface couplings, the velocity
// multigrid hierarchy (nested P2 spaces, rediscretized levels, vertex-patch smoother) and the
// operator's row blocks.
//
// Weak form (symmetric; the Darcy equation multiplied by -1):
//   a(u, v) = mu int grad u : grad v + alpha mu K^{-1/2} int_Gamma u_x v_x
//   b(v, q) = -int q div v,  c(v, q) = int_Gamma q v.nu = -int_Gamma q v_y,  d = K int grad . grad
//   [A_u  B^T  C    ] [u  ]
//   [B    0    0    ] [p_S]
//   [C^T  0    -K A_D] [p_D]
//
// Element integrals are exact: the gradients of the P2 basis (vertex lambda_i (2 lambda_i - 1),
// edge 4 lambda_i lambda_j) are linear in the barycentric coordinates, and products of those
// integrate by int lambda_i lambda_j = |T| (1 + delta_ij) / 12, int lambda_i = |T| / 3.
// Geometry comes from integer vertex offsets (scaled by h), so congruent triangles give
// bit-identical element matrices and congruent patches bit-identical patch matrices.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ds_internal.h"
#include "ell_host.h"

namespace fdd {

namespace {

// P2 velocity unknown of component c at half-grid node (A, B) on level m; -1 on the no-slip sides
inline int vidx(int m, int c, int A, int B) {
  if (A <= 0 || A >= 2 * m) return -1;
  return c * (2 * m - 1) * (2 * m + 1) + B * (2 * m - 1) + (A - 1);
}

// Triangle t of cell (ci, cj): t = 0 lower (v, v + (1, 0), v + (1, 1)), t = 1 upper
// (v, v + (1, 1), v + (0, 1)); local P2 nodes: vertices 0, 1, 2, midpoints 01, 12, 02.
struct P2Tri {
  int vi[3], vj[3];        // vertex grid coordinates
  int A[6], B[6];          // half-grid nodes
  double area;
  double G[3][2];          // barycentric gradients
  double S[6][6];          // int grad phi_a . grad phi_b
  double D[3][6][2];       // int lambda_k d_c phi_a
  double M1[3][3];         // int lambda_a lambda_b
  double A1[3][3];         // int grad lambda_a . grad lambda_b
};

P2Tri p2_triangle(int m, int ci, int cj, int t) {
  static const int off[2][3][2] = {{{0, 0}, {1, 0}, {1, 1}}, {{0, 0}, {1, 1}, {0, 1}}};
  static const int edge[3][2] = {{0, 1}, {1, 2}, {0, 2}};
  P2Tri T{};
  const double h = 1.0 / m;
  for (int a = 0; a < 3; ++a) {
    T.vi[a] = ci + off[t][a][0];
    T.vj[a] = cj + off[t][a][1];
    T.A[a] = 2 * T.vi[a];
    T.B[a] = 2 * T.vj[a];
  }
  for (int e = 0; e < 3; ++e) {
    T.A[3 + e] = T.vi[edge[e][0]] + T.vi[edge[e][1]];
    T.B[3 + e] = T.vj[edge[e][0]] + T.vj[edge[e][1]];
  }
  const double b00 = (off[t][1][0] - off[t][0][0]) * h, b10 = (off[t][1][1] - off[t][0][1]) * h;
  const double b01 = (off[t][2][0] - off[t][0][0]) * h, b11 = (off[t][2][1] - off[t][0][1]) * h;
  const double det = b00 * b11 - b01 * b10;
  T.G[1][0] = b11 / det;
  T.G[1][1] = -b01 / det;
  T.G[2][0] = -b10 / det;
  T.G[2][1] = b00 / det;
  T.G[0][0] = -(T.G[1][0] + T.G[2][0]);
  T.G[0][1] = -(T.G[1][1] + T.G[2][1]);
  T.area = std::fabs(det) / 2.0;
  // moments of (1, lambda_0, lambda_1, lambda_2)
  double mom[4][4];
  mom[0][0] = T.area;
  for (int i = 0; i < 3; ++i) {
    mom[0][1 + i] = mom[1 + i][0] = T.area / 3.0;
    for (int j = 0; j < 3; ++j) mom[1 + i][1 + j] = T.area * (i == j ? 2.0 : 1.0) / 12.0;
  }
  // grad phi_a = sum_k coef[a][k] . (1, lambda) G_k
  double coef[6][3][4] = {};
  for (int a = 0; a < 3; ++a) {
    coef[a][a][0] = -1.0;
    coef[a][a][1 + a] = 4.0;
  }
  for (int e = 0; e < 3; ++e) {
    const int i = edge[e][0], j = edge[e][1];
    coef[3 + e][j][1 + i] = 4.0;
    coef[3 + e][i][1 + j] = 4.0;
  }
  auto integral = [&](const double* p, const double* q) {
    double s = 0.0;
    for (int u = 0; u < 4; ++u)
      for (int v = 0; v < 4; ++v) s += p[u] * mom[u][v] * q[v];
    return s;
  };
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 6; ++b) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
          const double gg = T.G[k][0] * T.G[l][0] + T.G[k][1] * T.G[l][1];
          if (gg != 0.0) s += gg * integral(coef[a][k], coef[b][l]);
        }
      T.S[a][b] = s;
    }
  for (int k = 0; k < 3; ++k) {
    double lam[4] = {0, 0, 0, 0};
    lam[1 + k] = 1.0;
    for (int a = 0; a < 6; ++a)
      for (int c = 0; c < 2; ++c) {
        double s = 0.0;
        for (int q = 0; q < 3; ++q)
          if (T.G[q][c] != 0.0) s += T.G[q][c] * integral(lam, coef[a][q]);
        T.D[k][a][c] = s;
      }
  }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      T.M1[a][b] = T.area * (a == b ? 2.0 : 1.0) / 12.0;
      T.A1[a][b] = T.area * (T.G[a][0] * T.G[b][0] + T.G[a][1] * T.G[b][1]);
    }
  return T;
}

// P2 mass of one interface segment of length h (nodes: start, midpoint, end) / h
constexpr double kSegMass[3][3] = {{4.0 / 30, 2.0 / 30, -1.0 / 30},
                                   {2.0 / 30, 16.0 / 30, 2.0 / 30},
                                   {-1.0 / 30, 2.0 / 30, 4.0 / 30}};
// int (P1 hat at the start / end) x (P2 node function) over a segment / h
constexpr double kSegHat[2][3] = {{1.0 / 6, 1.0 / 3, 0.0}, {0.0, 1.0 / 3, 1.0 / 6}};

// a(., .) on level m into rb (rows and columns: velocity unknowns + col0)
void assemble_velocity(int m, double mu, double bjs, RowBuilder* rb, int col0) {
  for (int cj = 0; cj < m; ++cj)
    for (int ci = 0; ci < m; ++ci)
      for (int t = 0; t < 2; ++t) {
        const P2Tri T = p2_triangle(m, ci, cj, t);
        for (int c = 0; c < 2; ++c)
          for (int a = 0; a < 6; ++a) {
            const int ia = vidx(m, c, T.A[a], T.B[a]);
            if (ia < 0) continue;
            for (int b = 0; b < 6; ++b) {
              const int ib = vidx(m, c, T.A[b], T.B[b]);
              if (ib >= 0) rb->add(ia, col0 + ib, mu * T.S[a][b]);
            }
          }
      }
  if (bjs > 0.0) {
    const double h = 1.0 / m;
    for (int k = 0; k < m; ++k)
      for (int a = 0; a < 3; ++a) {
        const int ia = vidx(m, 0, 2 * k + a, 0);
        if (ia < 0) continue;
        for (int b = 0; b < 3; ++b) {
          const int ib = vidx(m, 0, 2 * k + b, 0);
          if (ib >= 0) rb->add(ia, col0 + ib, bjs * h * kSegMass[a][b]);
        }
      }
  }
}

// Prolongation from level m / 2 to level m (both components): a fine node's value of a coarse
// P2 function, evaluated in the coarse triangle holding it (all values are dyadic, so exact).
void build_prolongation(int m, HdLevel* fine) {
  const int mc = m / 2, nu = 2 * (2 * m - 1) * (2 * m + 1), nuc = 2 * (2 * mc - 1) * (2 * mc + 1);
  RowBuilder rb(nu, 6);
  for (int B = 0; B <= 2 * m; ++B)
    for (int A = 1; A < 2 * m; ++A) {
      const double X = A / 4.0, Y = B / 4.0;   // in coarse cells
      const int ci = std::min((int)std::floor(X), mc - 1), cj = std::min((int)std::floor(Y), mc - 1);
      const double lx = X - ci, ly = Y - cj;
      const int t = lx >= ly ? 0 : 1;
      double lam[3];
      if (t == 0) {
        lam[0] = 1.0 - lx;
        lam[1] = lx - ly;
        lam[2] = ly;
      } else {
        lam[0] = 1.0 - ly;
        lam[1] = lx;
        lam[2] = ly - lx;
      }
      const double phi[6] = {lam[0] * (2 * lam[0] - 1), lam[1] * (2 * lam[1] - 1),
                             lam[2] * (2 * lam[2] - 1), 4 * lam[0] * lam[1], 4 * lam[1] * lam[2],
                             4 * lam[0] * lam[2]};
      const P2Tri T = p2_triangle(mc, ci, cj, t);
      for (int c = 0; c < 2; ++c) {
        const int row = vidx(m, c, A, B);
        for (int a = 0; a < 6; ++a) {
          const int col = vidx(mc, c, T.A[a], T.B[a]);
          if (col >= 0 && phi[a] != 0.0) rb.add(row, col, phi[a]);
        }
      }
    }
  rb.to_ell(&fine->P, nuc);
  ell_transpose(fine->P, nuc, &fine->R);
}

// Vertex patches of level m: per component, the vertex's own node and the midpoints of its six
// edges (those not on the no-slip sides).
const char* velocity_patches(HdLevel* L) {
  const int m = L->n;
  static const int nb[7][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, -1}, {0, 1}, {-1, -1}, {1, 1}};
  const int nv = (m + 1) * (m + 1);
  return build_patch_tables(L, 2 * nv, 8, [&](int v, int* dofs) {
    const int c = v / nv, i = (v % nv) % (m + 1), j = (v % nv) / (m + 1);
    int k = 0;
    for (int q = 0; q < 7; ++q) {
      const int A = 2 * i + nb[q][0], B = 2 * j + nb[q][1];
      if (B < 0 || B > 2 * m) continue;
      const int d = vidx(m, c, A, B);
      if (d >= 0) dofs[k++] = d;
    }
    return k;
  });
}

// Darcy free dof of vertex (i, j) of the unit square (interior points row by row, Gamma = row n
// last), -1 on the Dirichlet boundary
inline int didx(int n, int i, int j) {
  if (i <= 0 || i >= n || j <= 0) return -1;
  return (j - 1) * (n - 1) + (i - 1);
}

}  // namespace

const char* ds_build(ProblemDS* D, int n, double K, double mu, double alpha, int krylov) {
  D->n = n;
  D->K = K;
  D->mu = mu;
  D->alpha = alpha;
  D->krylov = krylov;
  D->Nu = 2 * (2 * n - 1) * (2 * n + 1);
  D->Np = (n + 1) * (n + 1);
  D->ND = n * (n - 1);
  D->N = D->Nu + D->Np + D->ND;
  const double bjs = alpha * mu / std::sqrt(K);
  // velocity hierarchy
  int nl = 0;
  for (int m = n; m >= kDsCoarseN; m /= 2) {
    if (nl == kHdMaxLevels) return "too many levels";
    HdLevel& L = D->lev[nl++];
    L.n = m;
    L.n0 = 2 * (2 * m - 1) * (2 * m + 1);
    RowBuilder rb(L.n0, 20);
    assemble_velocity(m, mu, bjs, &rb, 0);
    if (rb.overflow) return "velocity assembly: more couplings per row than the mesh allows";
    rb.to_ell(&L.A, L.n0);
    if (const char* err = velocity_patches(&L)) return err;
  }
  D->nlev = nl;
  for (int l = 0; l + 1 < nl; ++l) build_prolongation(D->lev[l].n, &D->lev[l]);
  {
    const HdLevel& C = D->lev[nl - 1];
    std::vector<double> A((size_t)C.n0 * C.n0);
    for (int i = 0; i < C.n0; ++i)
      for (int j = 0; j < C.n0; ++j) A[(size_t)i * C.n0 + j] = ell_entry(C.A, i, j);
    if (!spd_inverse(A, C.n0)) return "the coarsest velocity matrix is not positive definite";
    D->cinv = A;
  }
  const int Nu = D->Nu, Np = D->Np, off = Nu + Np;
  const double h = 1.0 / n;
  // pressure mass with one-dof patches (Jacobi)
  {
    HdLevel& L = D->mass;
    L.n = n;
    L.n0 = Np;
    RowBuilder rb(Np, 7);
    for (int cj = 0; cj < n; ++cj)
      for (int ci = 0; ci < n; ++ci)
        for (int t = 0; t < 2; ++t) {
          const P2Tri T = p2_triangle(n, ci, cj, t);
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
              rb.add(T.vj[a] * (n + 1) + T.vi[a], T.vj[b] * (n + 1) + T.vi[b], T.M1[a][b]);
        }
    if (rb.overflow) return "pressure mass: more couplings per row than the mesh allows";
    rb.to_ell(&L.A, Np);
    if (const char* err = build_patch_tables(&L, Np, 1, [](int v, int* dofs) {
          dofs[0] = v;
          return 1;
        }))
      return err;
  }
  // operator rows: velocity [A_u B^T C], pressure [B], Darcy [C^T -K A_D]
  {
    RowBuilder ru(Nu, 28), rp(Np, 38), rd(D->ND, 12);
    assemble_velocity(n, mu, bjs, &ru, 0);
    for (int cj = 0; cj < n; ++cj)
      for (int ci = 0; ci < n; ++ci)
        for (int t = 0; t < 2; ++t) {
          const P2Tri T = p2_triangle(n, ci, cj, t);
          for (int c = 0; c < 2; ++c)
            for (int a = 0; a < 6; ++a) {
              const int ia = vidx(n, c, T.A[a], T.B[a]);
              if (ia < 0) continue;
              for (int k = 0; k < 3; ++k) {
                const int pk = T.vj[k] * (n + 1) + T.vi[k];
                const double v = -T.D[k][a][c];
                if (v == 0.0) continue;
                ru.add(ia, Nu + pk, v);
                rp.add(pk, ia, v);
              }
            }
          // Darcy stiffness on the same triangle of the unit square
          for (int a = 0; a < 3; ++a) {
            const int da = didx(n, T.vi[a], T.vj[a]);
            if (da < 0) continue;
            for (int b = 0; b < 3; ++b) {
              const int db = didx(n, T.vi[b], T.vj[b]);
              if (db >= 0 && T.A1[a][b] != 0.0) rd.add(da, off + db, -K * T.A1[a][b]);
            }
          }
        }
    // coupling c(v, q) = -int_Gamma q v_y on the segments of y = 1
    for (int k = 0; k < n; ++k)
      for (int a = 0; a < 3; ++a) {
        const int iy = vidx(n, 1, 2 * k + a, 0);
        if (iy < 0) continue;
        for (int e = 0; e < 2; ++e) {
          const int dq = didx(n, k + e, n);
          const double v = -h * kSegHat[e][a];
          if (dq < 0 || v == 0.0) continue;
          ru.add(iy, off + dq, v);
          rd.add(dq, iy, v);
        }
      }
    if (ru.overflow || rp.overflow || rd.overflow)
      return "operator assembly: more couplings per row than the mesh allows";
    ru.to_ell(&D->Au, D->N);
    rp.to_ell(&D->Bp, D->N);
    rd.to_ell(&D->Dd, D->N);
  }
  return nullptr;
}

size_t ds_plan(ProblemDS* D, char* base) {
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
  auto level = [&](HdLevel& L, bool transfers) {
    mat(L.A);
    if (transfers) {
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
  };
  for (int l = 0; l < D->nlev; ++l) level(D->lev[l], l + 1 < D->nlev);
  level(D->mass, false);
  D->dcinv = (double*)take(D->cinv.size() * 8);
  mat(D->Au);
  mat(D->Bp);
  mat(D->Dd);
  const size_t nu = (size_t)D->Nu * 8, np = (size_t)D->Np * 8, N = (size_t)D->N * 8;
  D->ur = (double*)take(nu);
  D->uz = (double*)take(nu);
  D->up = (double*)take(2 * nu);
  D->uq = (double*)take(nu);
  D->pz = (double*)take(np);
  D->pq = (double*)take(np);
  D->pp = (double*)take(np);
  const size_t m = (size_t)D->krylov;
  D->V = (double*)take((m + 1) * N);
  D->Z = (double*)take(m * N);
  D->Hm = (double*)take((m + 1) * m * 8);
  D->cs = (double*)take(m * 8);
  D->sn = (double*)take(m * 8);
  D->g = (double*)take((m + 1) * 8);
  D->y = (double*)take(m * 8);
  D->hp = (double*)take((m + 1) * 8);
  D->partials = (double*)take(std::max<size_t>((m + 1) * kDsChunks, 2 * kHdPartials) * 8);
  D->st_u = (HdState*)take(sizeof(HdState));
  D->st = (DsState*)take(sizeof(DsState));
  return (off + 255) / 256 * 256;
}

}  // namespace fdd
