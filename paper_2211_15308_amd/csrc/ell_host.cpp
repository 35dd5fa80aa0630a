// Host-side building blocks of the typed-ELL multigrid hierarchies (ell_host.h).
#include "ell_host.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <unordered_map>

namespace fdd {

bool RowBuilder::add(int i, int j, double v) {
  int* cs = &col[(size_t)i * cap];
  double* vs = &val[(size_t)i * cap];
  for (int k = 0; k < cnt[i]; ++k)
    if (cs[k] == j) {
      vs[k] += v;
      return true;
    }
  if (cnt[i] == cap) {
    overflow = true;
    return false;
  }
  cs[cnt[i]] = j;
  vs[cnt[i]] = v;
  ++cnt[i];
  return true;
}

void RowBuilder::to_ell(HdMat* M, int ncols) const {
  int w = 1;
  for (int i = 0; i < rows; ++i) w = std::max(w, cnt[i]);
  M->rows = rows;
  M->cols = ncols;
  M->width = w;
  M->col.assign((size_t)rows * w, 0);
  M->val.assign((size_t)rows * w, 0.0);
  M->rtype.assign(rows, 0);
  M->tval.clear();
  std::unordered_map<std::string, int> types;
  std::vector<std::pair<int, double>> tmp;
  std::vector<double> vals(w);
  for (int i = 0; i < rows; ++i) {
    tmp.clear();
    for (int k = 0; k < cnt[i]; ++k) tmp.emplace_back(col[(size_t)i * cap + k], val[(size_t)i * cap + k]);
    std::sort(tmp.begin(), tmp.end());
    for (int k = 0; k < w; ++k) {
      const bool used = k < (int)tmp.size();
      M->col[(size_t)k * rows + i] = used ? tmp[k].first : std::min(i, ncols - 1);
      vals[k] = used ? tmp[k].second : 0.0;
      M->val[(size_t)k * rows + i] = vals[k];
    }
    const std::string key((const char*)vals.data(), vals.size() * sizeof(double));
    auto it = types.find(key);
    int t;
    if (it == types.end()) {
      t = (int)types.size();
      types.emplace(key, t);
      M->tval.insert(M->tval.end(), vals.begin(), vals.end());
    } else {
      t = it->second;
    }
    M->rtype[i] = t;
  }
  M->ntypes = (int)types.size();
  M->toff.clear();
  // relative form: a type is the value sequence together with the column offsets col - i; kept
  // when at most kMaxRelTypes types arise and at least 64 rows share a type on average.  (Tables
  // of thousands of types, read per row with little locality, were measured slower than the
  // per-row columns: the H(div) levels keep the absolute form.)
  constexpr size_t kMaxRelTypes = 256;
  const size_t max_types = std::min<size_t>(kMaxRelTypes, (size_t)rows / 64);
  std::unordered_map<std::string, int> rel;
  std::vector<int> rtype(rows), toff;
  std::vector<double> rtval;
  std::vector<int> offs(w);
  std::string key;
  for (int i = 0; i < rows; ++i) {
    for (int k = 0; k < w; ++k) {
      vals[k] = M->val[(size_t)k * rows + i];
      offs[k] = M->col[(size_t)k * rows + i] - i;
    }
    key.assign((const char*)vals.data(), vals.size() * sizeof(double));
    key.append((const char*)offs.data(), offs.size() * sizeof(int));
    auto it = rel.find(key);
    if (it != rel.end()) {
      rtype[i] = it->second;
      continue;
    }
    if (rel.size() >= max_types) return;   // too many: keep the absolute columns
    const int t = (int)rel.size();
    rel.emplace(key, t);
    rtval.insert(rtval.end(), vals.begin(), vals.end());
    toff.insert(toff.end(), offs.begin(), offs.end());
    rtype[i] = t;
  }
  M->rtype = rtype;
  M->tval = rtval;
  M->toff = toff;
  M->ntypes = (int)rel.size();
}

double ell_entry(const HdMat& M, int i, int j) {
  for (int k = 0; k < M.width; ++k) {
    const size_t o = (size_t)k * M.rows + i;
    if (M.col[o] == j && M.val[o] != 0.0) return M.val[o];
  }
  return 0.0;
}

void ell_transpose(const HdMat& P, int cols, HdMat* R) {
  const int rows = P.rows;
  std::vector<int> cnt(cols, 0);
  for (int k = 0; k < P.width; ++k)
    for (int i = 0; i < rows; ++i)
      if (P.val[(size_t)k * rows + i] != 0.0) cnt[P.col[(size_t)k * rows + i]]++;
  int w = 1;
  for (int c : cnt) w = std::max(w, c);
  RowBuilder rt(cols, w);
  for (int i = 0; i < rows; ++i)
    for (int k = 0; k < P.width; ++k) {
      const double v = P.val[(size_t)k * rows + i];
      if (v != 0.0) rt.add(P.col[(size_t)k * rows + i], i, v);
    }
  rt.to_ell(R, rows);
}

bool spd_inverse(std::vector<double>& A, int m) {
  std::vector<double> L((size_t)m * m, 0.0);
  for (int j = 0; j < m; ++j) {
    double d = A[(size_t)j * m + j];
    for (int k = 0; k < j; ++k) d -= L[(size_t)j * m + k] * L[(size_t)j * m + k];
    if (!(d > 0)) return false;
    L[(size_t)j * m + j] = std::sqrt(d);
    for (int i = j + 1; i < m; ++i) {
      double v = A[(size_t)i * m + j];
      for (int k = 0; k < j; ++k) v -= L[(size_t)i * m + k] * L[(size_t)j * m + k];
      L[(size_t)i * m + j] = v / L[(size_t)j * m + j];
    }
  }
  // inverse column by column: L L^T x = e_c
  std::vector<double> inv((size_t)m * m), y(m);
  for (int c = 0; c < m; ++c) {
    for (int i = 0; i < m; ++i) {
      double v = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) v -= L[(size_t)i * m + k] * y[k];
      y[i] = v / L[(size_t)i * m + i];
    }
    for (int i = m - 1; i >= 0; --i) {
      double v = y[i];
      for (int k = i + 1; k < m; ++k) v -= L[(size_t)k * m + i] * inv[(size_t)k * m + c];
      inv[(size_t)i * m + c] = v / L[(size_t)i * m + i];
    }
  }
  A = inv;
  return true;
}

const char* build_patch_tables(HdLevel* L, int nvert, int pw,
                               const std::function<int(int, int*)>& list) {
  const int n0 = L->n0;
  if (pw != 1 && pw != 8 && pw != kHdPatch) return "patch stride must be 1, 8 or 12";
  L->nvert = nvert;
  L->pw = pw;
  L->patch.assign((size_t)nvert * pw, -1);
  L->ptype.assign(nvert, -1);
  L->slot.assign((size_t)n0 * 2, -1);
  std::vector<std::vector<double>> types;
  std::vector<int> tsize;
  for (int v = 0; v < nvert; ++v) {
    int dofs[kHdPatch];
    const int m = list(v, dofs);
    if (m == 0) continue;
    if (m > pw) return "a vertex patch has more dofs than the patch stride";
    std::sort(dofs, dofs + m);
    std::vector<double> A((size_t)m * m);
    for (int a = 0; a < m; ++a)
      for (int b = 0; b < m; ++b) A[(size_t)a * m + b] = ell_entry(L->A, dofs[a], dofs[b]);
    int t = -1;
    for (size_t q = 0; q < types.size() && t < 0; ++q)
      if (tsize[q] == m && std::memcmp(types[q].data(), A.data(), A.size() * sizeof(double)) == 0)
        t = (int)q;
    if (t < 0) {
      if ((int)types.size() == kHdMaxTypes) return "too many distinct vertex patches";
      types.push_back(A);
      tsize.push_back(m);
      t = (int)types.size() - 1;
    }
    L->ptype[v] = t;
    for (int a = 0; a < m; ++a) {
      L->patch[(size_t)v * pw + a] = dofs[a];
      int* s = &L->slot[(size_t)dofs[a] * 2];
      if (s[0] >= 0 && s[1] >= 0) return "a dof lies in more than two vertex patches";
      s[s[0] < 0 ? 0 : 1] = v * pw + a;
    }
  }
  L->ntypes = (int)types.size();
  L->pinv.assign((size_t)L->ntypes * pw * pw, 0.0);
  for (int t = 0; t < L->ntypes; ++t) {
    std::vector<double> A = types[t];
    const int m = tsize[t];
    if (!spd_inverse(A, m)) return "a vertex patch matrix is not positive definite";
    for (int a = 0; a < m; ++a)
      for (int b = 0; b < m; ++b)
        L->pinv[((size_t)t * pw + a) * pw + b] = A[(size_t)a * m + b];
  }
  return nullptr;
}

}  // namespace fdd
