// Host-side setup of the HHG library: macro-mesh validation and primitives, per-macro
// stencils from the macro geometry, Gauss-Seidel colourings, the level-0 factorisation and
// the workspace plan.  Nothing here touches the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <thread>

#include "hhg_internal.h"
#include "hhg_lattice.h"

namespace hhg {

int64_t tri_count(int64_t m) { return m < 0 ? 0 : (m + 1) * (m + 2) / 2; }
int64_t tet_count(int64_t m) { return m < 0 ? 0 : (m + 1) * (m + 2) * (m + 3) / 6; }
static int64_t lin2(int64_t n, int64_t i, int64_t j) { return j * (n + 1) - j * (j - 1) / 2 + i; }

int64_t lin_closure(int dim, int n, int i, int j, int k) {
  if (dim == 2) return lin2(n, i, j);
  int m = n - k;
  return tet_count(n) - tet_count(m) + lin2(m, i, j);
}

int zero_mask(int dim, int n, int i, int j, int k) {
  int c0 = n - i - j - (dim == 3 ? k : 0);
  int mk = (c0 == 0 ? 1 : 0) | (i == 0 ? 2 : 0) | (j == 0 ? 4 : 0);
  if (dim == 3 && k == 0) mk |= 8;
  return mk;
}

static int nprim(hhg_ctx c) { return (int)c->nV + c->nE + c->nF; }

// ---------------------------------------------------------------------------------------
// topology
static double simplex_det(int d, const double* x0, const double* x1, const double* x2, const double* x3) {
  if (d == 2) {
    double a = x1[0] - x0[0], b = x2[0] - x0[0], cc = x1[1] - x0[1], dd = x2[1] - x0[1];
    return a * dd - b * cc;
  }
  double a[3], b[3], e[3];
  for (int q = 0; q < 3; ++q) { a[q] = x1[q] - x0[q]; b[q] = x2[q] - x0[q]; e[q] = x3[q] - x0[q]; }
  return a[0] * (b[1] * e[2] - b[2] * e[1]) - a[1] * (b[0] * e[2] - b[2] * e[0]) + a[2] * (b[0] * e[1] - b[1] * e[0]);
}

hhg_status build_topology(hhg_ctx c) {
  const int d = c->dim, nv = d + 1;
  const int64_t nC = c->nC;
  for (int64_t m = 0; m < nC; ++m)
    for (int a = 0; a < nv; ++a) {
      int v = c->cells[m * nv + a];
      if (v < 0 || v >= c->nV) { c->err = "cell vertex id out of range"; return HHG_EMESH; }
      for (int b = 0; b < a; ++b)
        if (c->cells[m * nv + b] == v) { c->err = "cell with repeated vertex"; return HHG_EMESH; }
    }
  // degenerate cells
  double scale = 0.0;
  for (double x : c->coords) scale = std::max(scale, std::fabs(x));
  if (scale == 0.0) scale = 1.0;
  for (int64_t m = 0; m < nC; ++m) {
    const int* cv = &c->cells[m * nv];
    const double* X = c->coords.data();
    double det = simplex_det(d, X + cv[0] * d, X + cv[1] * d, X + cv[2] * d, d == 3 ? X + cv[3] * d : nullptr);
    if (!(std::fabs(det) > 1e-13 * std::pow(scale, d))) { c->err = "degenerate macro element " + std::to_string(m); return HHG_EMESH; }
  }
  // edges and faces
  std::map<std::array<int, 2>, int> emap;
  std::map<std::array<int, 3>, int> fmap;
  std::vector<std::array<int, 2>> E;
  std::vector<std::array<int, 3>> F;
  for (int64_t m = 0; m < nC; ++m) {
    const int* cv = &c->cells[m * nv];
    for (int a = 0; a < nv; ++a)
      for (int b = a + 1; b < nv; ++b) {
        std::array<int, 2> e{std::min(cv[a], cv[b]), std::max(cv[a], cv[b])};
        emap.emplace(e, 0);
      }
    if (d == 3)
      for (int s = 0; s < 4; ++s) {
        std::array<int, 3> f;
        int q = 0;
        for (int a = 0; a < 4; ++a) if (a != s) f[q++] = cv[a];
        std::sort(f.begin(), f.end());
        fmap.emplace(f, 0);
      }
  }
  for (auto& kv : emap) { kv.second = (int)E.size(); E.push_back(kv.first); }
  for (auto& kv : fmap) { kv.second = (int)F.size(); F.push_back(kv.first); }
  c->nE = (int)E.size();
  c->nF = (int)F.size();
  c->edges.resize(2 * E.size());
  for (size_t e = 0; e < E.size(); ++e) { c->edges[2 * e] = E[e][0]; c->edges[2 * e + 1] = E[e][1]; }
  c->faces.resize(3 * F.size());
  for (size_t f = 0; f < F.size(); ++f) for (int q = 0; q < 3; ++q) c->faces[3 * f + q] = F[f][q];

  const int NP = nprim(c);
  auto prim_of = [&](const std::vector<int>& sv) -> int {
    if (sv.size() == 1) return sv[0];
    if (sv.size() == 2) return (int)c->nV + emap.at({sv[0], sv[1]});
    return (int)c->nV + c->nE + fmap.at({sv[0], sv[1], sv[2]});
  };
  // facet adjacency counts -> boundary primitives
  std::vector<int> facet_count(d == 2 ? c->nE : c->nF, 0);
  for (int64_t m = 0; m < nC; ++m) {
    const int* cv = &c->cells[m * nv];
    for (int s = 0; s < nv; ++s) {
      std::vector<int> sv;
      for (int a = 0; a < nv; ++a) if (a != s) sv.push_back(cv[a]);
      std::sort(sv.begin(), sv.end());
      int p = prim_of(sv) - (int)c->nV - (d == 3 ? c->nE : 0);
      facet_count[p]++;
    }
  }
  std::vector<uint8_t> onb(NP, 0);
  for (size_t p = 0; p < facet_count.size(); ++p) {
    if (facet_count[p] > 2) { c->err = "non-manifold facet"; return HHG_EMESH; }
    if (facet_count[p] == 1) {
      std::vector<int> sv;
      if (d == 2) sv = {E[p][0], E[p][1]};
      else sv = {F[p][0], F[p][1], F[p][2]};
      // all sub-primitives of the facet lie on the boundary
      int k = (int)sv.size();
      for (int sub = 1; sub < (1 << k); ++sub) {
        std::vector<int> t;
        for (int q = 0; q < k; ++q) if (sub & (1 << q)) t.push_back(sv[q]);
        onb[prim_of(t)] = 1;
      }
    }
  }
  c->primdir.assign(NP, 0);
  for (int p = 0; p < NP; ++p) {
    if (!onb[p]) continue;
    if (c->vdir_user.empty()) { c->primdir[p] = 1; continue; }
    std::vector<int> sv;
    if (p < c->nV) sv = {p};
    else if (p < c->nV + c->nE) sv = {E[p - c->nV][0], E[p - c->nV][1]};
    else sv = {F[p - c->nV - c->nE][0], F[p - c->nV - c->nE][1], F[p - c->nV - c->nE][2]};
    bool all = true;
    for (int v : sv) all = all && c->vdir_user[v];
    c->primdir[p] = all ? 1 : 0;
  }
  // incidences and per-macro sub-primitive tables
  std::vector<std::vector<Inc>> plist(NP);
  c->subprim.assign(nC * kMaxMask, -1);
  c->suborder.assign(nC * kMaxMask, 0);
  c->dirbits.assign(nC, 0);
  c->ownbits.assign(nC, 0);
  const int full = (1 << nv) - 1;
  for (int64_t m = 0; m < nC; ++m) {
    const int* cv = &c->cells[m * nv];
    for (int keep = 1; keep < full; ++keep) {   // set of local slots that span the primitive
      std::vector<std::pair<int, int>> vs;      // (global id, slot)
      for (int a = 0; a < nv; ++a) if (keep & (1 << a)) vs.push_back({cv[a], a});
      std::sort(vs.begin(), vs.end());
      std::vector<int> sv;
      for (auto& pr : vs) sv.push_back(pr.first);
      int p = prim_of(sv);
      int mask = full & ~keep;
      Inc in{};
      in.macro = (int32_t)m;
      uint8_t packed = 0;
      for (size_t r = 0; r < vs.size(); ++r) { in.slot[r] = (uint8_t)vs[r].second; packed |= (uint8_t)(vs[r].second << (2 * r)); }
      in.mask = (uint8_t)mask;
      plist[p].push_back(in);
      c->subprim[m * kMaxMask + mask] = p;
      c->suborder[m * kMaxMask + mask] = packed;
      if (c->primdir[p]) c->dirbits[m] |= (uint16_t)(1u << mask);
    }
  }
  c->inc_off.assign(NP + 1, 0);
  c->inc.clear();
  for (int p = 0; p < NP; ++p) {
    // macro ids ascend because macros were visited in order
    c->inc_off[p] = (int32_t)c->inc.size();
    for (auto& in : plist[p]) c->inc.push_back(in);
    if (!plist[p].empty()) {
      const Inc& own = plist[p][0];
      c->ownbits[own.macro] |= (uint16_t)(1u << own.mask);
    }
  }
  c->inc_off[NP] = (int32_t)c->inc.size();
  // dyadic scale for red-black parity
  c->dyadic_p = -1;
  for (int p = 0; p <= 40 && c->dyadic_p < 0; ++p) {
    bool ok = true;
    double s = std::ldexp(1.0, p);
    for (double x : c->coords) { double y = x * s; if (y != std::floor(y) || std::fabs(y) > 9.0e15) { ok = false; break; } }
    if (ok) c->dyadic_p = p;
  }
  c->rbpar.assign(nC * 4, 0);
  if (c->dyadic_p >= 0) {
    double s = std::ldexp(1.0, c->dyadic_p);
    for (int64_t m = 0; m < nC; ++m) {
      const int* cv = &c->cells[m * nv];
      long long x0s = 0;
      for (int q = 0; q < d; ++q) x0s += (long long)(c->coords[cv[0] * d + q] * s);
      c->rbpar[m * 4 + 0] = (int)(((x0s % 2) + 2) % 2);
      for (int a = 1; a < nv; ++a) {
        long long sa = 0;
        for (int q = 0; q < d; ++q) sa += (long long)((c->coords[cv[a] * d + q] - c->coords[cv[0] * d + q]) * s);
        c->rbpar[m * 4 + a] = (int)(((sa % 2) + 2) % 2);
      }
    }
  }
  return HHG_OK;
}

// ---------------------------------------------------------------------------------------
// stencils
static void element_matrices(int d, const double y[4][3], double K[4][4], double Mm[4][4]) {
  double J[3][3] = {{0}}, G[3][3] = {{0}};
  for (int a = 0; a < d; ++a)
    for (int q = 0; q < d; ++q) J[q][a] = y[a + 1][q] - y[0][q];   // columns y_a - y_0
  double det;
  if (d == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    G[0][0] = J[1][1] / det; G[0][1] = -J[0][1] / det;
    G[1][0] = -J[1][0] / det; G[1][1] = J[0][0] / det;
  } else {
    det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
          J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    G[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    G[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    G[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    G[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    G[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    G[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    G[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    G[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    G[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  }
  // rows of G = J^{-1} are the gradients of lambda_1..lambda_d
  double g[4][3] = {{0}};
  for (int a = 0; a < d; ++a)
    for (int q = 0; q < d; ++q) { g[a + 1][q] = G[a][q]; g[0][q] -= G[a][q]; }
  double vol = std::fabs(det) / (d == 2 ? 2.0 : 6.0);
  for (int a = 0; a <= d; ++a)
    for (int b = 0; b <= d; ++b) {
      double s = 0;
      for (int q = 0; q < d; ++q) s += g[a][q] * g[b][q];
      K[a][b] = vol * s;
      Mm[a][b] = vol * (a == b ? 2.0 : 1.0) / ((d + 1) * (d + 2));
    }
}

static bool dir_valid(int dim, int mask, int di, int dj, int dk) {
  int dc[4] = {-(di + dj + dk), di, dj, dk};
  if (dim == 2) dc[0] = -(di + dj);
  for (int q = 0; q <= dim; ++q)
    if ((mask >> q) & 1)
      if (dc[q] < 0) return false;
  return true;
}

hhg_status build_stencils(hhg_ctx c) {
  const int d = c->dim, nv = d + 1;
  const int ND = d == 3 ? kNDir3 : kNDir2, NT = d == 3 ? kNType3 : kNType2;
  const int64_t nC = c->nC;
  c->validdirs.assign(kMaxMask, 0);
  for (int mask = 0; mask < kMaxMask; ++mask)
    for (int q = 0; q < ND; ++q) {
      int di = d == 3 ? kOff3[q][0] : kOff2[q][0];
      int dj = d == 3 ? kOff3[q][1] : kOff2[q][1];
      int dk = d == 3 ? kOff3[q][2] : 0;
      if (dir_valid(d, mask, di, dj, dk)) c->validdirs[mask] |= (uint16_t)(1u << q);
    }
  // valid incident (type, vertex) pairs per mask: every other element vertex offset valid
  c->incvalid.assign(kMaxMask, 0);
  for (int mask = 0; mask < kMaxMask; ++mask)
    for (int t = 0; t < NT; ++t)
      for (int a = 0; a < nv; ++a) {
        bool ok = true;
        for (int b = 0; b < nv; ++b) {
          int o[3] = {0, 0, 0};
          for (int q = 0; q < d; ++q) o[q] = (d == 3 ? kType3[t][b][q] - kType3[t][a][q] : kType2[t][b][q] - kType2[t][a][q]);
          ok = ok && dir_valid(d, mask, o[0], o[1], o[2]);
        }
        if (ok) c->incvalid[mask] |= (1u << (t * nv + a));
      }
  c->stiff.assign(nC * kMaxMask * ND, 0.0);
  c->mass.assign(nC * kMaxMask * ND, 0.0);
  c->elemK.assign(nC * NT * nv * nv, 0.0);
  for (int64_t m = 0; m < nC; ++m) {
    const int* cv = &c->cells[m * nv];
    double X[4][3] = {{0}};
    for (int a = 0; a < nv; ++a) for (int q = 0; q < d; ++q) X[a][q] = c->coords[cv[a] * d + q];
    for (int t = 0; t < NT; ++t) {
      double y[4][3] = {{0}};
      for (int a = 0; a < nv; ++a)
        for (int q = 0; q < d; ++q) {
          double v = X[0][q];
          for (int s = 0; s < d; ++s) {
            int o = d == 3 ? kType3[t][a][s] : kType2[t][a][s];
            v += o * (X[s + 1][q] - X[0][q]);
          }
          y[a][q] = v;
        }
      double K[4][4], Mm[4][4];
      element_matrices(d, y, K, Mm);
      for (int a = 0; a < nv; ++a)
        for (int b = 0; b < nv; ++b) c->elemK[((m * NT + t) * nv + a) * nv + b] = K[a][b];
      for (int mask = 0; mask < kMaxMask; ++mask)
        for (int a = 0; a < nv; ++a) {
          if (!((c->incvalid[mask] >> (t * nv + a)) & 1)) continue;
          for (int b = 0; b < nv; ++b) {
            int o[3] = {0, 0, 0};
            for (int q = 0; q < d; ++q) o[q] = (d == 3 ? kType3[t][b][q] - kType3[t][a][q] : kType2[t][b][q] - kType2[t][a][q]);
            int di = d == 3 ? dir_index3(o[0], o[1], o[2]) : dir_index2(o[0], o[1]);
            c->stiff[(m * kMaxMask + mask) * ND + di] += K[a][b];
            c->mass[(m * kMaxMask + mask) * ND + di] += Mm[a][b];
          }
        }
    }
    // snap round-off couplings (right angles give exact zeros in exact arithmetic)
    double mx = 0;
    for (int q = 0; q < kMaxMask * ND; ++q) mx = std::max(mx, std::fabs(c->stiff[m * kMaxMask * ND + q]));
    for (int q = 0; q < kMaxMask * ND; ++q)
      if (std::fabs(c->stiff[m * kMaxMask * ND + q]) < 1e-14 * mx) c->stiff[m * kMaxMask * ND + q] = 0.0;
    for (int q = 0; q < NT * nv * nv; ++q)
      if (std::fabs(c->elemK[m * NT * nv * nv + q]) < 1e-14 * mx) c->elemK[m * NT * nv * nv + q] = 0.0;
  }
  // red-black exactness: every nonzero off-centre coupling must change the parity
  if (c->opt.smoother == HHG_GS_REDBLACK) {
    if (c->dyadic_p < 0) { c->err = "red-black colouring needs dyadic coordinates"; return HHG_EINVAL; }
    for (int64_t m = 0; m < nC; ++m)
      for (int t = 0; t < NT; ++t)
        for (int a = 0; a < nv; ++a)
          for (int b = 0; b < nv; ++b) {
            if (a == b || c->elemK[((m * NT + t) * nv + a) * nv + b] == 0.0) continue;
            int par = 0;
            for (int q = 0; q < d; ++q) {
              int o = d == 3 ? kType3[t][b][q] - kType3[t][a][q] : kType2[t][b][q] - kType2[t][a][q];
              par += o * c->rbpar[m * 4 + 1 + q];
            }
            if (((par % 2) + 2) % 2 == 0) {
              c->err = "red-black Gauss-Seidel is not exact on macro " + std::to_string(m) +
                       " (same-colour coupling); use HHG_GS_MULTICOLOR";
              return HHG_EINVAL;
            }
          }
  }
  return HHG_OK;
}

// ---------------------------------------------------------------------------------------
// canonical numbering and colouring
int64_t canonical_index(hhg_ctx c, const Level& lv, int m, int i, int j, int k) {
  const int d = c->dim, n = lv.n;
  int mask = zero_mask(d, n, i, j, k);
  if (mask == 0) {
    int64_t li = lin_closure(d, n - d - 1, i - 1, j - 1, k - 1);
    return lv.nIface + (int64_t)m * lv.NI + li;
  }
  int p = c->subprim[m * kMaxMask + mask];
  uint8_t ord = c->suborder[m * kMaxMask + mask];
  int cc[4] = {n - i - j - (d == 3 ? k : 0), i, j, k};
  if (p < c->nV) return p;
  if (p < c->nV + c->nE) {
    int a = cc[(ord >> 2) & 3];
    return c->nV + (int64_t)(p - c->nV) * lv.nEd + (a - 1);
  }
  int a = cc[(ord >> 2) & 3], b = cc[(ord >> 4) & 3];
  return c->nV + (int64_t)c->nE * lv.nEd + (int64_t)(p - c->nV - c->nE) * lv.nFd + lin2(n - 3, a - 1, b - 1);
}

// interface DoF t -> primitive and coordinates along the primitive's sorted vertices
static void iface_decode(hhg_ctx c, const Level& lv, int64_t t, int& p, int co[3]) {
  const int n = lv.n;
  co[0] = co[1] = co[2] = 0;
  if (t < c->nV) { p = (int)t; co[0] = n; return; }
  t -= c->nV;
  if (t < (int64_t)c->nE * lv.nEd) {
    p = c->nV + (int)(t / lv.nEd);
    int a = (int)(t % lv.nEd) + 1;
    co[0] = n - a; co[1] = a;
    return;
  }
  t -= (int64_t)c->nE * lv.nEd;
  p = c->nV + c->nE + (int)(t / lv.nFd);
  int64_t s = t % lv.nFd;
  int side = n - 3, b = 0;
  while (lin2(side, 0, b + 1) <= s && b + 1 <= side) ++b;
  int a = (int)(s - lin2(side, 0, b));
  co[1] = a + 1; co[2] = b + 1; co[0] = n - co[1] - co[2];
}

static int interior_colour(hhg_ctx c, int l, int m, int i, int j, int k) {
  if (c->opt.smoother == HHG_JACOBI) return 0;
  if (c->opt.smoother == HHG_GS_REDBLACK) {
    const int* rp = &c->rbpar[m * 4];
    int s = (l == 0 ? rp[0] : 0) + i * rp[1] + j * rp[2] + (c->dim == 3 ? k * rp[3] : 0);
    return s & 1;
  }
  return c->dim == 2 ? (i + 2 * j) % 3 : (i + 2 * j + 3 * k) % 4;
}

// 2D Gauss-Seidel: an edge point at distance a (2 <= a <= n - 2) from the edge's lower-id
// vertex sweeps in class Cint + (a mod 2); it touches only interior points, its own edge and
// the vertex neighbourhoods (a = 1, a = n - 1, macro vertices), which follow from Cint + 2
static bool edge_class_2d(hhg_ctx c, const Level& lv, int p, const int co[3]) {
  return c->dim == 2 && c->opt.smoother != HHG_JACOBI && p >= c->nV && p < c->nV + c->nE && co[1] >= 2 &&
         co[1] <= lv.n - 2;
}

hhg_status build_colouring(hhg_ctx c) {
  // Sweep order: macro-interior colour classes 0..Cint-1, then interface classes Cint, ...
  // (2D: the two edge classes Cint, Cint + 1, then the vertex neighbourhoods from Cint + 2)
  const int d = c->dim;
  const int ND = d == 3 ? kNDir3 : kNDir2;
  const int Cint = c->opt.smoother == HHG_JACOBI ? 1 : (c->opt.smoother == HHG_GS_REDBLACK ? 2 : (d == 2 ? 3 : 4));
  const int Cvr = d == 2 && c->opt.smoother != HHG_JACOBI ? Cint + 2 : Cint;
  // 2D edge records of the edge-class sweep (kEdgeRecWords words per macro edge; the
  // coefficients are filled in at upload, fill_kappa_tables)
  c->erec.clear();
  bool erec_ok = d == 2 && c->opt.smoother != HHG_JACOBI && c->opt.coefficient == HHG_KAPPA_MACRO;
  if (erec_ok) {
    c->erec.assign((size_t)c->nE * kEdgeRecWords, 0);
    for (int64_t e = 0; e < c->nE && erec_ok; ++e) {
      const int p = (int)(c->nV + e);
      const int cnt = c->inc_off[p + 1] - c->inc_off[p];
      if (cnt < 1 || cnt > 2) { erec_ok = false; break; }
      int32_t* Rr = &c->erec[(size_t)e * kEdgeRecWords];
      Rr[0] = cnt | (c->primdir[p] ? 4 : 0);
      for (int k = 0; k < cnt; ++k) {
        const Inc& in = c->inc[c->inc_off[p] + k];
        if (in.macro < 0 || in.macro >= c->nC || in.slot[0] > 2 || in.slot[1] > 2 || in.mask >= kMaxMask) {
          erec_ok = false;
          break;
        }
        int32_t* Cc = Rr + 2 + kEdgeCopyWords * k;
        Cc[0] = in.macro;
        Cc[1] = in.slot[0] | (in.slot[1] << 8) | (in.mask << 16);
        double* KW = reinterpret_cast<double*>(Cc + 2);
        for (int dd = 0; dd < kNDir2; ++dd) KW[1 + dd] = c->stiff[((size_t)in.macro * kMaxMask + in.mask) * kNDir2 + dd];
        Cc[18] = (int32_t)c->validdirs[in.mask];
      }
    }
    if (!erec_ok) c->erec.clear();
  }
  for (auto& lv : c->lev) {
    std::vector<int> col(lv.nIface, -1);
    for (int64_t t = 0; t < lv.nIface; ++t) {
      int p, co[3];
      iface_decode(c, lv, t, p, co);
      if (c->primdir[p]) continue;
      const Inc& in0 = c->inc[c->inc_off[p]];
      int cc[4] = {0, 0, 0, 0};
      int np = p < c->nV ? 1 : (p < c->nV + c->nE ? 2 : 3);
      for (int r = 0; r < np; ++r) cc[in0.slot[r]] = co[r];
      if (c->opt.smoother == HHG_JACOBI) { col[t] = Cint; continue; }
      if (edge_class_2d(c, lv, p, co)) { col[t] = Cint + (co[1] & 1); continue; }
      if (c->opt.smoother == HHG_GS_REDBLACK) {
        col[t] = Cvr + interior_colour(c, lv.l, in0.macro, cc[1], cc[2], cc[3]);
        continue;
      }
      // greedy first fit against the neighbours of the same kind coloured so far (2D: vertex
      // neighbourhoods only; the edge classes lie below Cvr)
      uint64_t used = 0;
      for (int q = c->inc_off[p]; q < c->inc_off[p + 1]; ++q) {
        const Inc& in = c->inc[q];
        int lc[4] = {0, 0, 0, 0};
        for (int r = 0; r < np; ++r) lc[in.slot[r]] = co[r];
        for (int dd = 1; dd < ND; ++dd) {
          if (!((c->validdirs[in.mask] >> dd) & 1)) continue;
          int i2 = lc[1] + (d == 3 ? kOff3[dd][0] : kOff2[dd][0]);
          int j2 = lc[2] + (d == 3 ? kOff3[dd][1] : kOff2[dd][1]);
          int k2 = d == 3 ? lc[3] + kOff3[dd][2] : 0;
          if (zero_mask(d, lv.n, i2, j2, k2) == 0) continue;
          const int cn = col[canonical_index(c, lv, in.macro, i2, j2, k2)];
          if (cn >= 0 && cn < 64) used |= (1ull << cn);
        }
      }
      int cnew = Cvr;
      while ((used >> cnew) & 1) ++cnew;
      col[t] = cnew;
    }
    int maxc = -1;
    for (int v : col) maxc = std::max(maxc, v);
    // Dirichlet interface DoFs join the first interface class: their update only rewrites
    // their own (fixed) value, into both iterate buffers of the out-of-place 2D sweep
    for (int64_t t = 0; t < lv.nIface; ++t) {
      int p, co[3];
      iface_decode(c, lv, t, p, co);
      if (c->primdir[p]) col[t] = Cint;
    }
    maxc = std::max(maxc, lv.nIface > 0 ? Cint : -1);
    lv.interior_colours = Cint;
    lv.ncolours = std::max(Cint, maxc + 1);
    lv.interior_per_colour.assign(Cint, 0);
    if (lv.NI > 0) {
      const int n = lv.n;
      for (int64_t m = 0; m < c->nC; ++m)
        for (int k = (d == 3 ? 1 : 0); k <= (d == 3 ? n - 3 : 0); ++k)
          for (int j = 1; j <= n - 2 - (d == 3 ? k : 0); ++j)
            for (int i = 1; i <= n - 1 - j - (d == 3 ? k : 0); ++i)
              lv.interior_per_colour[interior_colour(c, lv.l, (int)m, i, j, k)]++;
    }
    lv.colour_off.assign(lv.ncolours + 1, 0);
    for (int v : col) if (v >= 0) lv.colour_off[v + 1]++;
    for (int q = 0; q < lv.ncolours; ++q) lv.colour_off[q + 1] += lv.colour_off[q];
    lv.max_iface_class = 0;
    for (int q = Cint; q < lv.ncolours; ++q)
      lv.max_iface_class = std::max(lv.max_iface_class, lv.colour_off[q + 1] - lv.colour_off[q]);
    lv.colour_list.assign(lv.colour_off[lv.ncolours], 0);
    std::vector<int32_t> fill(lv.colour_off.begin(), lv.colour_off.end() - 1);
    for (int64_t t = 0; t < lv.nIface; ++t)
      if (col[t] >= 0) lv.colour_list[fill[col[t]]++] = (int32_t)t;
    // lane-parallel interface tasks (Gauss-Seidel with a per-macro coefficient): every
    // non-empty interface class packed into wavefronts, a DoF's lanes never split; every
    // entry is checked here (copy index inside the level vector, coordinates inside the
    // closure), so the kernel only follows validated indices
    lv.task_ok = false;
    lv.task_copy.clear(); lv.task_info.clear(); lv.task_loc.clear(); lv.task_seg.clear(); lv.task_wmax.clear();
    lv.task_woff.assign(lv.ncolours + 1, 0);
    if (c->opt.smoother != HHG_JACOBI && c->opt.coefficient == HHG_KAPPA_MACRO && lv.nfull < (int64_t)1 << 29 &&
        c->nC < (1 << 24) && lv.n < 2048) {
      bool ok = true;
      auto pad_wave = [&]() {
        while (lv.task_copy.size() % 64) {
          lv.task_copy.push_back(-1); lv.task_info.push_back(0); lv.task_loc.push_back(0); lv.task_seg.push_back(0);
        }
      };
      const int np_of[3] = {1, 2, 3};
      for (int cc = 0; cc < lv.ncolours && ok; ++cc) {
        lv.task_woff[cc] = (int32_t)(lv.task_copy.size() / 64);
        for (int32_t kk = lv.colour_off[cc]; kk < lv.colour_off[cc + 1] && ok; ++kk) {
          int p, co[3];
          iface_decode(c, lv, lv.colour_list[kk], p, co);
          const int q0 = c->inc_off[p], q1 = c->inc_off[p + 1], cnt = q1 - q0;
          if (cnt < 1 || cnt > 64) { ok = false; break; }
          const int np = np_of[p < c->nV ? 0 : (p < c->nV + c->nE ? 1 : 2)];
          if (lv.task_copy.size() % 64 + cnt > 64) pad_wave();
          const int lead = (int)(lv.task_copy.size() % 64);
          for (int q = q0; q < q1; ++q) {
            const Inc& in = c->inc[q];
            int lc[4] = {0, 0, 0, 0};
            for (int r = 0; r < np; ++r) lc[in.slot[r]] = co[r];
            const int i = lc[1], j = lc[2], k = lc[3];
            const int64_t loc = lin_closure(d, lv.n, i, j, k);
            if (i < 0 || j < 0 || k < 0 || i + j + k > lv.n || loc < 0 || loc >= lv.Sraw || in.macro < 0 ||
                in.macro >= c->nC || in.mask >= kMaxMask || zero_mask(d, lv.n, i, j, k) != in.mask) {
              ok = false;
              break;
            }
            lv.task_copy.push_back((int32_t)(in.macro * lv.S + loc));
            lv.task_info.push_back(in.macro | (in.mask << 24) | ((c->primdir[p] ? 1 : 0) << 28));
            lv.task_loc.push_back(i | (j << 11) | (k << 22));
            lv.task_seg.push_back(lead | (cnt << 8));
          }
        }
        pad_wave();
      }
      if (ok) {
        lv.task_woff[lv.ncolours] = (int32_t)(lv.task_copy.size() / 64);
        const int nw = lv.task_woff[lv.ncolours];
        lv.task_wmax.assign(nw, 0);
        for (int w = 0; w < nw; ++w)
          for (int q = 0; q < 64; ++q) lv.task_wmax[w] = std::max(lv.task_wmax[w], lv.task_seg[w * 64 + q] >> 8);
        lv.task_ok = true;
      } else {
        lv.task_copy.clear(); lv.task_info.clear(); lv.task_loc.clear(); lv.task_seg.clear();
        lv.task_woff.assign(lv.ncolours + 1, 0);
      }
    }
    // 2D levels whose edge classes are too large for the single-workgroup interface sweep:
    // both edge classes in one launch by edge chunks (at most two incident macros per edge, at
    // most 16 chunks), which also copies the Dirichlet vertex values; indices checked here
    lv.fused_iface = false;
    lv.dvcopy.clear();
    lv.c_vr0 = Cint + 2;
    if (d == 2 && lv.task_ok && erec_ok && lv.n >= 4 && lv.n <= 1024 && lv.ncolours >= Cint + 2) {
      bool ok = true;
      for (int64_t v = 0; v < c->nV && ok; ++v) {
        if (!c->primdir[v]) continue;
        for (int q = c->inc_off[v]; q < c->inc_off[v + 1]; ++q) {
          const Inc& in = c->inc[q];
          int lc[3] = {0, 0, 0};
          lc[in.slot[0]] = lv.n;
          const int64_t loc = lin_closure(2, lv.n, lc[1], lc[2], 0);
          if (in.macro < 0 || in.macro >= c->nC || loc < 0 || loc >= lv.Sraw) { ok = false; break; }
          lv.dvcopy.push_back((int32_t)(in.macro * lv.S + loc));
        }
      }
      lv.fused_iface = ok;
      if (!ok) lv.dvcopy.clear();
    }
    // the vertex classes of such a level by vertex neighbourhoods ("wheels"): a macro vertex
    // and the edge points next to it (a = 1 from it) touch no other vertex neighbourhood when
    // n >= 4, so one wavefront sweeps all vertex classes of a wheel in order, passing new
    // values between lanes; a wheel's lanes (one per copy of each DoF, DoFs in class order)
    // never split across wavefronts
    lv.wheels = false;
    lv.wh_merge = false;
    lv.wh_copy.clear(); lv.wh_info.clear(); lv.wh_loc.clear(); lv.wh_seg.clear(); lv.wh_src.clear();
    lv.wh_wmax.clear(); lv.wh_cw.clear(); lv.wh_e2.clear(); lv.wh_a2i.clear(); lv.wh_a2w.clear();
    if (lv.fused_iface && lv.ncolours - lv.c_vr0 <= 15) {
      bool ok = true;
      const int n = lv.n;
      std::vector<int> ev0(c->nE), ev1(c->nE);
      std::vector<std::vector<int>> vedges(c->nV);
      for (int64_t e = 0; e < c->nE; ++e) {
        const Inc& in = c->inc[c->inc_off[c->nV + e]];
        ev0[e] = c->cells[in.macro * 3 + in.slot[0]];
        ev1[e] = c->cells[in.macro * 3 + in.slot[1]];
        vedges[ev0[e]].push_back((int)e);
        vedges[ev1[e]].push_back((int)e);
      }
      // lead lane (within its wavefront) of every interface DoF placed so far, -1 otherwise
      std::vector<int> lead_of(lv.nIface, -1), wheel_of(lv.nIface, -1);
      int64_t placed = 0;
      for (int v = 0; v < c->nV && ok; ++v) {
        std::vector<int64_t> dofs;
        if (!c->primdir[v]) dofs.push_back(v);
        for (int e : vedges[v]) {
          if (c->primdir[c->nV + e]) continue;
          const int a = v == ev0[e] ? 1 : n - 1;
          dofs.push_back(c->nV + (int64_t)e * lv.nEd + (a - 1));
        }
        for (int64_t t : dofs)
          if (col[t] < lv.c_vr0) ok = false;
        if (!ok || dofs.empty()) continue;
        std::sort(dofs.begin(), dofs.end(), [&](int64_t x, int64_t y) { return col[x] != col[y] ? col[x] < col[y] : x < y; });
        int lanes = 0;
        for (int64_t t : dofs) {
          int p, co[3];
          iface_decode(c, lv, t, p, co);
          lanes += c->inc_off[p + 1] - c->inc_off[p];
        }
        if (lanes > 64) { ok = false; break; }
        if ((int)(lv.wh_copy.size() % 64) + lanes > 64)
          while (lv.wh_copy.size() % 64) {
            lv.wh_copy.push_back(-1); lv.wh_info.push_back(0); lv.wh_loc.push_back(0); lv.wh_seg.push_back(0);
          }
        for (int64_t t : dofs) {
          int p, co[3];
          iface_decode(c, lv, t, p, co);
          const int lead = (int)(lv.wh_copy.size() % 64), cnt = c->inc_off[p + 1] - c->inc_off[p];
          lead_of[t] = lead;
          wheel_of[t] = v;
          const int np = p < c->nV ? 1 : 2;
          for (int q = c->inc_off[p]; q < c->inc_off[p + 1]; ++q) {
            const Inc& in = c->inc[q];
            int lc[4] = {0, 0, 0, 0};
            for (int r = 0; r < np; ++r) lc[in.slot[r]] = co[r];
            const int64_t loc = lin_closure(2, n, lc[1], lc[2], 0);
            if (loc < 0 || loc >= lv.Sraw || zero_mask(2, n, lc[1], lc[2], 0) != in.mask) { ok = false; break; }
            lv.wh_copy.push_back((int32_t)(in.macro * lv.S + loc));
            lv.wh_info.push_back(in.macro | (in.mask << 24) | ((col[t] - lv.c_vr0) << 28));
            lv.wh_loc.push_back(lc[1] | (lc[2] << 11));
            lv.wh_seg.push_back(lead | (cnt << 8));
          }
        }
        placed += (int64_t)dofs.size();
      }
      // every vertex-class DoF sits in exactly one wheel
      int64_t nvr = 0;
      for (int64_t t = 0; t < lv.nIface; ++t)
        if (col[t] >= lv.c_vr0) ++nvr;
      if (placed != nvr) ok = false;
      while (lv.wh_copy.size() % 64) {
        lv.wh_copy.push_back(-1); lv.wh_info.push_back(0); lv.wh_loc.push_back(0); lv.wh_seg.push_back(0);
      }
      // per lane and direction: the lane holding that neighbour if it is a DoF of the same
      // wheel (0xff otherwise: read from memory); no vertex-class neighbour may lie outside.
      // A neighbour in an edge class (at most one per lane: a = 2 from the wheel's vertex on
      // the lane's own edge) is recorded for the one-launch form, which recomputes it
      bool merge = true;
      for (size_t idx = 0; idx < lv.wh_copy.size() && ok; ++idx) {
        uint32_t sa = 0xffffffffu, sb = 0xffffffffu;
        int32_t e2 = -1;
        if (lv.wh_copy[idx] >= 0) {
          const int m = lv.wh_info[idx] & 0xffffff, mask = (lv.wh_info[idx] >> 24) & 15;
          const int i = lv.wh_loc[idx] & 2047, j = lv.wh_loc[idx] >> 11;
          // the DoF of this lane
          const int64_t tself = canonical_index(c, lv, m, i, j, 0);
          for (int dd = 1; dd < kNDir2; ++dd) {
            if (!((c->validdirs[mask] >> dd) & 1)) continue;
            const int i2 = i + kOff2[dd][0], j2 = j + kOff2[dd][1];
            if (zero_mask(2, n, i2, j2, 0) == 0) continue;
            const int64_t tn = canonical_index(c, lv, m, i2, j2, 0);
            if (tn < 0 || tn >= lv.nIface) { ok = false; break; }
            if (col[tn] < lv.c_vr0) {   // edge class or Dirichlet: from memory
              int p2, co2[3];
              iface_decode(c, lv, tn, p2, co2);
              if (p2 >= c->nV && p2 < c->nV + c->nE && !c->primdir[p2]) {
                const int a2 = co2[1];
                if (e2 >= 0 || (a2 != 2 && a2 != n - 2) || (c->nE >= (1 << 24))) merge = false;
                else e2 = (p2 - (int)c->nV) | ((a2 == 2 ? 0 : 1) << 24) | (dd << 25);
              }
              continue;
            }
            if (wheel_of[tn] != wheel_of[tself] || lead_of[tn] < 0) { ok = false; break; }
            const uint32_t sl = (uint32_t)lead_of[tn];
            if (dd <= 4) sa = (sa & ~(0xffu << (8 * (dd - 1)))) | (sl << (8 * (dd - 1)));
            else sb = (sb & ~(0xffu << (8 * (dd - 5)))) | (sl << (8 * (dd - 5)));
          }
        }
        lv.wh_src.push_back((int32_t)sa);
        lv.wh_src.push_back((int32_t)sb);
        lv.wh_e2.push_back(e2);
      }
      // per lane: the macro's coefficient (filled in at upload) and its unit stencil weights
      // for the lane's mask, as a struct of arrays
      const size_t nl = lv.wh_copy.size();
      lv.wh_cw.assign(nl * (kNDir2 + 1), 0.0);
      for (size_t idx = 0; idx < nl; ++idx) {
        if (lv.wh_copy[idx] < 0) continue;
        const int m = lv.wh_info[idx] & 0xffffff, mask = (lv.wh_info[idx] >> 24) & 15;
        for (int dd = 0; dd < kNDir2; ++dd) lv.wh_cw[(1 + dd) * nl + idx] = c->stiff[((size_t)m * kMaxMask + mask) * kNDir2 + dd];
      }
      const int nw = (int)(lv.wh_copy.size() / 64);
      lv.wh_wmax.assign(nw, 0);
      for (int w = 0; w < nw; ++w)
        for (int q = 0; q < 64; ++q) lv.wh_wmax[w] = std::max(lv.wh_wmax[w], lv.wh_seg[w * 64 + q] >> 8);
      lv.wheels = ok;
      lv.wh_merge = ok && merge && !c->erec.empty();
      if (lv.wh_merge) {
        // the rows of each lane's edge-class neighbour, from the edge records (the coefficient
        // is filled in with the others, fill_kappa_tables)
        lv.wh_a2i.assign(nl * 16, -1);
        lv.wh_a2w.assign(nl * 16, 0.0);
        for (size_t idx = 0; idx < nl && lv.wh_merge; ++idx) {
          const int32_t e2 = lv.wh_e2[idx];
          if (e2 < 0) continue;
          const int e = e2 & 0xffffff, a = ((e2 >> 24) & 1) ? n - 2 : 2;
          const int32_t* Rr = &c->erec[(size_t)e * kEdgeRecWords];
          const int ncp = Rr[0] & 3;
          for (int k = 0; k < ncp && k < 2; ++k) {
            const int32_t* Cc = Rr + 2 + kEdgeCopyWords * k;
            const int macro = Cc[0], sl = Cc[1];
            const int s0 = sl & 3, s1 = (sl >> 8) & 3, mask = (sl >> 16) & 15;
            int lc[3] = {0, 0, 0};
            lc[s0] = n - a;
            lc[s1] = a;
            const int64_t base = (int64_t)macro * lv.S;
            const int64_t cpk = base + lin_closure(2, n, lc[1], lc[2], 0);
            if (cpk < 0 || cpk >= lv.nfull) { lv.wh_merge = false; break; }
            lv.wh_a2i[(size_t)(8 * k) * nl + idx] = (int32_t)cpk;
            int fl = 0;
            for (int dd = 1; dd < kNDir2; ++dd) {
              if (!((c->validdirs[mask] >> dd) & 1)) continue;
              const int i2 = lc[1] + kOff2[dd][0], j2 = lc[2] + kOff2[dd][1];
              const int64_t ix = base + lin_closure(2, n, i2, j2, 0);
              if (i2 < 0 || j2 < 0 || i2 + j2 > n || ix < base || ix >= base + lv.Sraw) { lv.wh_merge = false; break; }
              lv.wh_a2i[(size_t)(8 * k + dd) * nl + idx] = (int32_t)ix;
              if (zero_mask(2, n, i2, j2, 0) != 0) fl |= 1 << (dd - 1);
            }
            lv.wh_a2i[(size_t)(8 * k + 7) * nl + idx] = fl;
            for (int dd = 0; dd < kNDir2; ++dd)
              lv.wh_a2w[(size_t)(8 * k + 1 + dd) * nl + idx] = c->stiff[((size_t)macro * kMaxMask + mask) * kNDir2 + dd];
          }
        }
      }
      if (!lv.wh_merge) { lv.wh_e2.clear(); lv.wh_a2i.clear(); lv.wh_a2w.clear(); }
      if (!ok) {
        lv.wh_copy.clear(); lv.wh_info.clear(); lv.wh_loc.clear(); lv.wh_seg.clear(); lv.wh_src.clear();
        lv.wh_wmax.clear(); lv.wh_cw.clear();
      }
    }
    // tables of the fused interior sweeps
    lv.tiles.clear();
    lv.itab.clear();
    if (d == 2 && lv.NI > 0) {
      const int TI = 64 - 2 * Cint;   // one wavefront per tile of the fused sweep
      const int TJ = tile_rows(Cint, lv.n);
      for (int tj = 0; 1 + tj * TJ <= lv.n - 2; ++tj)
        for (int ti = 0; 1 + ti * TI + 1 + tj * TJ <= lv.n - 1; ++ti) lv.tiles.push_back(ti | (tj << 16));
    }
    // 3D red-black with a per-macro coefficient: plane-streaming tiles (i0, j0, k0 in units of
    // kS3I, kS3J, kS3K) of the levels with n >= kStream3dMinN, or of all levels with n >= 4
    // under HHG_FLAG_STREAM3D
    // (red-black colour alternating along i on every macro: the kernel pairs neighbouring points)
    bool alt_i = true;
    for (int64_t m = 0; m < c->nC && d == 3; ++m) alt_i = alt_i && (c->rbpar[m * 4 + 1] & 1) != 0;
    const bool rbmacro = d == 3 && lv.NI > 0 && c->opt.smoother == HHG_GS_REDBLACK &&
                         c->opt.coefficient == HHG_KAPPA_MACRO;
    const bool stream3d = rbmacro && alt_i && (lv.n >= kStream3dMinN || (c->force_stream3d && lv.n >= 4));
    // whole-plane sweep: the interior planes 1 .. n-3 of every macro in chunks [k0, k1) of about
    // equal cost (points of the chunk's planes plus the four planes read around it), as many
    // chunks per macro as make about kPlane3dBlocks workgroups, each at least 8 planes high
    lv.planes3d = rbmacro && !stream3d && !c->no_planes3d && lv.n <= kPlane3dMaxN &&
                  (lv.n >= kPlane3dMinN || (c->force_planes3d && lv.n >= 16));
    if (lv.planes3d) {
      const int n = lv.n, np = n - 3;
      auto psz = [&](int k) { return (double)(n - k + 1) * (n - k + 2) / 2.0; };
      const int nch = (int)std::max<int64_t>(1, std::min<int64_t>((kPlane3dBlocks + c->nC - 1) / c->nC, np / 8));
      double total = 0.0;
      for (int k = 1; k <= np; ++k) total += psz(k);
      int k0 = 1;
      double acc = 0.0;
      for (int k = 1; k <= np; ++k) {
        acc += psz(k);
        const int left = nch - (int)lv.tiles.size() - 1;   // chunks still to cut after this one
        if (k == np || (left > 0 && acc + 4.0 * psz(k0) >= total / nch && k - k0 + 1 >= 8 && np - k >= 8)) {
          lv.tiles.push_back(k0 | ((k + 1) << 16));
          k0 = k + 1;
          acc = 0.0;
        }
      }
    }
    if (stream3d) {
      for (int tk = 0; 1 + tk * kS3K <= lv.n - 3; ++tk)
        for (int tj = 0; 1 + tj * kS3J + 1 + tk * kS3K <= lv.n - 2; ++tj)
          for (int ti = 0; 1 + ti * kS3I + 1 + tj * kS3J + 1 + tk * kS3K <= lv.n - 1; ++ti)
            lv.tiles.push_back(ti | (tj << 10) | (tk << 20));
    }
    lv.itab_off.clear();
    if (d == 3 && lv.NI > 0 && lv.n <= kMacroLdsN && !stream3d && !lv.planes3d) {
      // interior points sorted by colour, one list per red-black parity pattern (s1, s2, s3)
      // of a macro (multicolour: one list); itab_off[p * (Cint + 1) + c] starts colour c
      const int n = lv.n;
      const bool rbs = c->opt.smoother == HHG_GS_REDBLACK;
      const int npat = rbs ? 8 : 1;
      for (int pat = 0; pat < npat; ++pat) {
        std::vector<std::vector<uint32_t>> bycol(Cint);
        for (int k = 1; k <= n - 3; ++k)
          for (int j = 1; j <= n - 2 - k; ++j)
            for (int i = 1; i <= n - 1 - j - k; ++i) {
              const int col = rbs ? ((i * (pat & 1) + j * ((pat >> 1) & 1) + k * ((pat >> 2) & 1)) & 1)
                                  : (Cint == 4 ? (i + 2 * j + 3 * k) % 4 : 0);
              bycol[col].push_back((uint32_t)i | ((uint32_t)j << 10) | ((uint32_t)k << 20));
            }
        int32_t o = 0;
        for (int cc = 0; cc < Cint; ++cc) {
          lv.itab_off.push_back(o);
          lv.itab.insert(lv.itab.end(), bycol[cc].begin(), bycol[cc].end());
          o += (int32_t)bycol[cc].size();
        }
        lv.itab_off.push_back(o);
      }
    }
  }
  return HHG_OK;
}

// ---------------------------------------------------------------------------------------
// level 0: exact solve on the inner coarse vertices.  Up to kCoarseDenseMax of them: the
// explicit inverse of the inner block (one matrix-vector product per solve).  More (the
// coarse mesh of a kl loop grows with every k-step): the inner block is renumbered by reverse
// Cuthill-McKee, factored P A P^T = L L^T by an envelope Cholesky (the fill stays inside the
// profile of the renumbered matrix), and the solve applies x = P^T X^T X P r with X = L^{-1},
// a dense lower triangle computed column by column on the host threads.
hhg_status build_coarse(hhg_ctx c, const double* kappa_vertex) {
  const int d = c->dim, nv = d + 1;
  std::vector<int> idx(c->nV, -1);
  c->coarse_vertex.clear();
  for (int v = 0; v < c->nV; ++v)
    if (!c->primdir[v]) { idx[v] = (int)c->coarse_vertex.size(); c->coarse_vertex.push_back(v); }
  const int n0 = (int)c->coarse_vertex.size();
  c->n0 = n0;
  const Level& l0 = c->lev[0];
  c->coarse_copy_off.assign(n0 + 1, 0);
  c->coarse_copy.clear();
  for (int r = 0; r < n0; ++r) {
    int v = c->coarse_vertex[r];
    c->coarse_copy_off[r] = (int32_t)c->coarse_copy.size();
    for (int q = c->inc_off[v]; q < c->inc_off[v + 1]; ++q) {
      const Inc& in = c->inc[q];
      c->coarse_copy.push_back((int64_t)in.macro * l0.S + in.slot[0]);   // at n = 1, lin == slot
    }
  }
  c->coarse_copy_off[n0] = (int32_t)c->coarse_copy.size();
  c->coarse_factored = n0 > kCoarseDenseMax;
  c->coarse_perm.assign(n0, 0);
  std::iota(c->coarse_perm.begin(), c->coarse_perm.end(), 0);
  c->Ainv.assign((size_t)n0 * n0, 0.0);
  if (n0 == 0) return HHG_OK;
  // inner block of A_0, row by row (sparse)
  std::vector<std::map<int, double>> rows(n0);
  for (int64_t m = 0; m < c->nC; ++m) {
    const int* cv = &c->cells[m * nv];
    double y[4][3] = {{0}};
    for (int a = 0; a < nv; ++a) for (int q = 0; q < d; ++q) y[a][q] = c->coords[cv[a] * d + q];
    double K[4][4], Mm[4][4];
    element_matrices(d, y, K, Mm);
    double kap = c->kappa_cell[m];
    if (c->opt.coefficient == HHG_KAPPA_P1) {
      kap = 0;
      for (int a = 0; a < nv; ++a) kap += kappa_vertex ? kappa_vertex[cv[a]] : 1.0;
      kap /= nv;
    }
    for (int a = 0; a < nv; ++a)
      for (int b = 0; b < nv; ++b) {
        int ra = idx[cv[a]], rb = idx[cv[b]];
        if (ra >= 0 && rb >= 0) rows[ra][rb] += kap * K[a][b];
      }
  }
  const char* spd = "level-0 matrix is not positive definite (no Dirichlet boundary?)";
  if (!c->coarse_factored) {
    std::vector<double> A((size_t)n0 * n0, 0.0);
    for (int r = 0; r < n0; ++r)
      for (const auto& kv : rows[r]) A[(size_t)r * n0 + kv.first] = kv.second;
    // Cholesky A = R^T R (upper R stored in A), then inverse column by column
    for (int k = 0; k < n0; ++k) {
      const double akk = A[(size_t)k * n0 + k];
      double s = akk;
      for (int q = 0; q < k; ++q) s -= A[(size_t)q * n0 + k] * A[(size_t)q * n0 + k];
      if (!(s > 1e-10 * akk)) { c->err = spd; return HHG_EINVAL; }
      double rkk = std::sqrt(s);
      A[(size_t)k * n0 + k] = rkk;
      for (int j = k + 1; j < n0; ++j) {
        double t = A[(size_t)k * n0 + j];
        for (int q = 0; q < k; ++q) t -= A[(size_t)q * n0 + k] * A[(size_t)q * n0 + j];
        A[(size_t)k * n0 + j] = t / rkk;
      }
    }
    std::vector<double> y(n0), x(n0);
    for (int col = 0; col < n0; ++col) {
      // R^T y = e_col
      for (int i = 0; i < n0; ++i) {
        double t = (i == col) ? 1.0 : 0.0;
        for (int q = 0; q < i; ++q) t -= A[(size_t)q * n0 + i] * y[q];
        y[i] = t / A[(size_t)i * n0 + i];
      }
      // R x = y
      for (int i = n0 - 1; i >= 0; --i) {
        double t = y[i];
        for (int q = i + 1; q < n0; ++q) t -= A[(size_t)i * n0 + q] * x[q];
        x[i] = t / A[(size_t)i * n0 + i];
      }
      for (int i = 0; i < n0; ++i) c->Ainv[(size_t)i * n0 + col] = x[i];
    }
    return HHG_OK;
  }
  // reverse Cuthill-McKee: breadth-first from a low-degree start vertex of every component,
  // neighbours by increasing degree, order reversed; perm[p] = inner vertex at position p
  std::vector<int> deg(n0), order;
  order.reserve(n0);
  for (int r = 0; r < n0; ++r) deg[r] = (int)rows[r].size();
  std::vector<char> seen(n0, 0);
  std::vector<int> byDeg(n0);
  std::iota(byDeg.begin(), byDeg.end(), 0);
  std::stable_sort(byDeg.begin(), byDeg.end(), [&](int x, int y) { return deg[x] < deg[y]; });
  for (int start : byDeg) {
    if (seen[start]) continue;
    size_t head = order.size();
    order.push_back(start);
    seen[start] = 1;
    while (head < order.size()) {
      const int r = order[head++];
      std::vector<int> nb;
      for (const auto& kv : rows[r])
        if (!seen[kv.first]) { nb.push_back(kv.first); seen[kv.first] = 1; }
      std::stable_sort(nb.begin(), nb.end(), [&](int x, int y) { return deg[x] < deg[y]; });
      order.insert(order.end(), nb.begin(), nb.end());
    }
  }
  std::reverse(order.begin(), order.end());
  std::vector<int> pos(n0);
  for (int p = 0; p < n0; ++p) { c->coarse_perm[p] = order[p]; pos[order[p]] = p; }
  // envelope of the renumbered matrix: row i holds columns f[i] .. i of L
  std::vector<int> f(n0);
  std::vector<int64_t> rs(n0 + 1, 0);
  for (int i = 0; i < n0; ++i) {
    int fi = i;
    for (const auto& kv : rows[order[i]]) fi = std::min(fi, pos[kv.first]);
    f[i] = fi;
    rs[i + 1] = rs[i] + (i - fi + 1);
  }
  std::vector<double> Lv(rs[n0], 0.0);
  auto L = [&](int i, int j) -> double& { return Lv[rs[i] + (j - f[i])]; };
  for (int i = 0; i < n0; ++i)
    for (const auto& kv : rows[order[i]]) {
      const int j = pos[kv.first];
      if (j <= i) L(i, j) = kv.second;
    }
  // up-looking envelope Cholesky
  for (int i = 0; i < n0; ++i) {
    for (int j = f[i]; j < i; ++j) {
      double t = L(i, j);
      for (int k = std::max(f[i], f[j]); k < j; ++k) t -= L(i, k) * L(j, k);
      L(i, j) = t / L(j, j);
    }
    const double aii = L(i, i);
    double t = aii;
    for (int k = f[i]; k < i; ++k) t -= L(i, k) * L(i, k);
    if (!(t > 1e-10 * aii)) { c->err = spd; return HHG_EINVAL; }
    L(i, i) = std::sqrt(t);
  }
  // X = L^{-1}, column-major (X[col * n0 + row], zero above the diagonal): column c solves
  // L x = e_c; the columns are independent and split over the host threads
  double* X = c->Ainv.data();
  auto columns = [&](int c0, int c1) {
    for (int col = c0; col < c1; ++col) {
      double* x = X + (size_t)col * n0;
      x[col] = 1.0 / L(col, col);
      for (int i = col + 1; i < n0; ++i) {
        double t = 0.0;
        for (int k = std::max(f[i], col); k < i; ++k) t += L(i, k) * x[k];
        x[i] = -t / L(i, i);
      }
    }
  };
  const int nt = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  // columns near the start cost the most (longest solves): deal them out round-robin in blocks
  std::vector<std::vector<std::pair<int, int>>> work(nt);
  const int blk = 16;
  for (int c0 = 0, t = 0; c0 < n0; c0 += blk, t = (t + 1) % nt) work[t].push_back({c0, std::min(n0, c0 + blk)});
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&, t]() {
      for (auto& r : work[t]) columns(r.first, r.second);
    });
  for (auto& th : pool) th.join();
  return HHG_OK;
}

// Level of the dense coarse map: the largest k <= L - 3 (L - 1 when forced) whose inner DoFs
// and map bytes fit the limits.  Its rows, and its columns, are the inner (non-Dirichlet) DoFs
// of level k in canonical order, each with the level-vector indices of its copies.
void build_dense_plan(hhg_ctx c) {
  c->dense_k = -1;
  c->dense_rows = c->dense_ld = c->dense_kmax = 0;
  c->dense_off.clear();
  c->dense_copy.clear();
  c->dense_gat.clear();
  if (c->no_dense) return;
  const int d = c->dim;
  for (int k = c->force_dense ? c->L - 1 : c->L - 3; k >= 1; --k) {
    const Level& lv = c->lev[k];
    const int n = lv.n;
    if (lv.ndof > 4 * (int64_t)kDenseMaxRows) continue;   // far too large: not worth counting
    std::vector<std::vector<int32_t>> copies(lv.ndof);
    for (int64_t m = 0; m < c->nC; ++m)
      for (int kk = 0; kk <= (d == 3 ? n : 0); ++kk)
        for (int j = 0; j <= n - kk; ++j)
          for (int i = 0; i <= n - kk - j; ++i) {
            const int mask = zero_mask(d, n, i, j, kk);
            if (mask != 0 && ((c->dirbits[m] >> mask) & 1)) continue;
            const int64_t t = canonical_index(c, lv, (int)m, i, j, kk);
            copies[t].push_back((int32_t)(m * lv.S + lin_closure(d, n, i, j, kk)));
          }
    int64_t rows = 0;
    size_t kmax = 0;
    for (const auto& v : copies) {
      rows += v.empty() ? 0 : 1;
      kmax = std::max(kmax, v.size());
    }
    const int64_t ld = (rows + 255) / 256 * 256;
    if (rows == 0 || rows > kDenseMaxRows || kmax > (size_t)kDenseMaxCopies || rows * ld * 12 > kDenseMaxBytes)
      continue;
    c->dense_off.push_back(0);
    for (const auto& v : copies) {
      if (v.empty()) continue;
      c->dense_copy.insert(c->dense_copy.end(), v.begin(), v.end());
      c->dense_off.push_back((int32_t)c->dense_copy.size());
    }
    // the gather table: copy q of row r at [q][r] as level-vector index + 1 (0: none)
    c->dense_kmax = (int)kmax;
    c->dense_gat.assign(kmax * (size_t)rows, 0);
    for (int64_t r = 0; r < rows; ++r)
      for (int32_t q = c->dense_off[r]; q < c->dense_off[r + 1]; ++q)
        c->dense_gat[(size_t)(q - c->dense_off[r]) * rows + r] = c->dense_copy[q] + 1;
    c->dense_k = k;
    c->dense_rows = (int)rows;
    c->dense_ld = (int)ld;
    return;
  }
}

// the per-macro coefficients inside the edge records and the wheel lane tables
void fill_kappa_tables(hhg_ctx c) {
  for (int64_t e = 0; e < (int64_t)(c->erec.size() / kEdgeRecWords); ++e) {
    int32_t* Rr = &c->erec[(size_t)e * kEdgeRecWords];
    for (int k = 0; k < (Rr[0] & 3); ++k) {
      int32_t* Cc = Rr + 2 + kEdgeCopyWords * k;
      reinterpret_cast<double*>(Cc + 2)[0] = c->kappa_cell[Cc[0]];
    }
  }
  for (auto& lv : c->lev) {
    for (size_t idx = 0; idx < lv.wh_copy.size(); ++idx)
      if (lv.wh_copy[idx] >= 0) lv.wh_cw[idx] = c->kappa_cell[lv.wh_info[idx] & 0xffffff];
    // the coefficients of the recomputed edge-class neighbours (copy k's macro from the edge
    // record of the lane's edge)
    const size_t nl = lv.wh_copy.size();
    if (lv.wh_a2w.size() == nl * 16)
      for (size_t idx = 0; idx < nl; ++idx) {
        const int32_t e2 = lv.wh_e2[idx];
        if (e2 < 0) continue;
        const int32_t* Rr = &c->erec[(size_t)(e2 & 0xffffff) * kEdgeRecWords];
        for (int k = 0; k < (Rr[0] & 3) && k < 2; ++k)
          lv.wh_a2w[(size_t)(8 * k) * nl + idx] = c->kappa_cell[Rr[2 + kEdgeCopyWords * k]];
      }
  }
}

// ---------------------------------------------------------------------------------------
// workspace plan
static int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

void plan_workspace(hhg_ctx c) {
  const int d = c->dim, nv = d + 1;
  const int ND = d == 3 ? kNDir3 : kNDir2, NT = d == 3 ? kNType3 : kNType2;
  int64_t off = 0;
  auto take = [&](int64_t bytes) { int64_t o = off; off = align256(off + std::max<int64_t>(bytes, 1)); return o; };
  const int64_t nC = c->nC;
  c->o_stiff = take(nC * kMaxMask * ND * 8);
  c->o_mass = take(nC * kMaxMask * ND * 8);
  c->o_elemK = take(nC * NT * nv * nv * 8);
  c->o_kappa = take(nC * 8);
  c->o_subprim = take(nC * kMaxMask * 4);
  c->o_suborder = take(nC * kMaxMask);
  c->o_dirbits = take(nC * 2);
  c->o_ownbits = take(nC * 2);
  c->o_rbpar = take(nC * 16);
  c->o_incoff = take((int64_t)c->inc_off.size() * 4);
  c->o_inc = take((int64_t)c->inc.size() * sizeof(Inc));
  c->o_primdir = take((int64_t)c->primdir.size());
  c->o_ccopyoff = take((int64_t)(c->n0 + 1) * 4);
  c->o_ccopy = take((int64_t)c->coarse_copy.size() * 8 + 8);
  c->o_ainv = take((int64_t)c->n0 * c->n0 * 8 + 8);
  c->o_cperm = take((int64_t)c->n0 * 4 + 4);
  c->o_cscr = take((int64_t)c->n0 * 2 * 8 + 16);
  c->o_dense32 = take((int64_t)c->dense_rows * c->dense_ld * 4);
  c->o_dense64 = take((int64_t)c->dense_rows * c->dense_ld * 8);
  c->o_doff = take((int64_t)c->dense_off.size() * 4);
  c->o_dcopy = take((int64_t)c->dense_copy.size() * 4);
  c->o_dgat = take((int64_t)c->dense_gat.size() * 4);
  c->o_dsum = take((int64_t)c->dense_rows * 8);
  // reduction scratch: per macro per block (4 values) on the finest level, and per block norms
  const Level& lt = c->lev[c->L];
  int64_t bpm = (lt.Sraw + 255) / 256;
  int64_t nblk_norm = nC * ((lt.NI + 255) / 256) + (lt.nIface + 255) / 256 + 16;
  c->red_capacity = std::max<int64_t>(std::max<int64_t>(nC * bpm * 4, nblk_norm), kNormBlocks + (lt.nIface + 255) / 256) + 1024;
  if (d == 2) {
    // the 2D row estimator: two sums per wavefront, kEstRows x 62 interior nodes or 64
    // boundary nodes of one macro per wavefront; its per-macro results follow the partials
    const int64_t n = lt.n;
    const int64_t wpm = ((n - 2 + kEstRows - 1) / kEstRows) * ((n - 2 + 61) / 62) + (3 * n + 63) / 64;
    c->red_capacity = std::max<int64_t>(c->red_capacity, nC * wpm * 2 + 2 * nC + 1024);
  }
  c->o_red = take(c->red_capacity * 8);
  c->o_scal = take(64 * 8);
  c->o_erec = take((int64_t)c->erec.size() * 4);
  c->o_mxyz = take(nC * nv * d * 8);
  c->o_aux0 = take(lt.nfull * 8);
  c->o_aux1 = take(lt.nfull * 8);
  for (auto& lv : c->lev) {
    const int64_t nf = lv.nfull;
    lv.off_x = take(nf * 8);
    lv.off_t = take(nf * 8);
    lv.off_bf = take(nf * 8);
    lv.off_rc = take(nf * 8);
    lv.off_g = take(nf * 8);
    lv.off_w = take(nf * 8);
    lv.off_kn = c->opt.coefficient == HHG_KAPPA_P1 ? take(nf * 8) : -1;
    lv.off_x32 = take(nf * 4);
    lv.off_t32 = take(nf * 4);
    lv.off_b32 = take(nf * 4);
    lv.off_cl = take((int64_t)lv.colour_list.size() * 4);
    lv.off_tiles = take((int64_t)lv.tiles.size() * 4);
    lv.off_coff = take((int64_t)lv.colour_off.size() * 4);
    lv.off_tcopy = take((int64_t)lv.task_copy.size() * 4);
    lv.off_tinfo = take((int64_t)lv.task_info.size() * 4);
    lv.off_tloc = take((int64_t)lv.task_loc.size() * 4);
    lv.off_tseg = take((int64_t)lv.task_seg.size() * 4);
    lv.off_twmax = take((int64_t)lv.task_wmax.size() * 4);
    lv.off_twoff = take((int64_t)lv.task_woff.size() * 4);
    lv.off_dvcopy = take((int64_t)lv.dvcopy.size() * 4);
    lv.off_whcw = take((int64_t)lv.wh_cw.size() * 8);
    lv.off_whe2 = take((int64_t)lv.wh_e2.size() * 4);
    lv.off_wha2i = take((int64_t)lv.wh_a2i.size() * 4);
    lv.off_wha2w = take((int64_t)lv.wh_a2w.size() * 8);
    lv.off_whcopy = take((int64_t)lv.wh_copy.size() * 4);
    lv.off_whinfo = take((int64_t)lv.wh_info.size() * 4);
    lv.off_whloc = take((int64_t)lv.wh_loc.size() * 4);
    lv.off_whseg = take((int64_t)lv.wh_seg.size() * 4);
    lv.off_whsrc = take((int64_t)lv.wh_src.size() * 4);
    lv.off_whwmax = take((int64_t)lv.wh_wmax.size() * 4);
    // second iterate buffers of the out-of-place fused sweeps (2D, and 3D with streaming tiles)
    lv.off_x2 = take(d == 2 || !lv.tiles.empty() ? nf * 8 : 0);
    lv.off_x2_32 = take(d == 2 || !lv.tiles.empty() ? nf * 4 : 0);
    lv.off_itab = take((int64_t)lv.itab.size() * 4);
    lv.off_itoff = take((int64_t)lv.itab_off.size() * 4);
  }
  c->ws_bytes = (size_t)off;
}

}  // namespace hhg
