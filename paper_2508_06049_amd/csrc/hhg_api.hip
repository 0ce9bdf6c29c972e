// C ABI of the HHG library and the host-side multigrid driver.
//
// The driver sequences kernel launches on the bound stream:
//   FMG (Algorithm 4, procedure FMG): level-0 exact solve, then for l = 1..L the prolongation
//   of the level-(l-1) solution (stored as w_{l-1}, Dirichlet data written on the boundary)
//   followed by nu V(pre,post) cycles; optional extra cycles on level L.
//   FP32_REFINED: every cycle is  r = b - A u (float64, stored float32), a float32 V-cycle on
//   the correction from zero, u += e (float64).  Level 0 is solved in float64 in both modes.
//   ErrorEstimate (Algorithm 4): one fused kernel over level L forms u_L - w_{L-1} and
//   u_L - P w_{L-2} and their per-macro mass norms.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hhg_internal.h"
#include "hhg_kernels.h"
#include "hhg_lattice.h"

using namespace hhg;

namespace {

thread_local std::string g_err;

#define HIPCHK(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      c->err = std::string(#call) + ": " + hipGetErrorString(e_);                 \
      return HHG_EHIP;                                                            \
    }                                                                             \
  } while (0)

#define LAUNCHCHK()                                                               \
  do {                                                                            \
    hipError_t e_ = hipGetLastError();                                            \
    if (e_ != hipSuccess) {                                                       \
      c->err = std::string("kernel launch: ") + hipGetErrorString(e_);            \
      return HHG_EHIP;                                                            \
    }                                                                             \
  } while (0)

#define TRY(x)                       \
  do {                               \
    hhg_status s_ = (x);             \
    if (s_ != HHG_OK) return s_;     \
  } while (0)

inline hipStream_t ST(hhg_ctx c) { return (hipStream_t)(c->capturing ? c->cap_stream : c->stream); }

LK lk_of(hhg_ctx c, int l) {
  const Level& lv = c->lev[l];
  LK k;
  k.n = lv.n;
  k.l = lv.l;
  k.S = lv.S;
  k.Sraw = (int)lv.Sraw;
  k.NI = (int)lv.NI;
  k.nEd = (int)lv.nEd;
  k.nFd = (int)lv.nFd;
  k.nIface = lv.nIface;
  k.ndof = lv.ndof;
  k.nmacro = (int)c->nC;
  // one wavefront per 3D lattice row pays off once rows are long (below n = 128 most lanes of
  // a wavefront would idle and the one-thread-per-point kernels are used)
  k.rows3d_min = c->force_rows3d ? 1 : 128;
  k.planes3d = lv.planes3d ? 1 : 0;
  return k;
}

// stiffness scales like n^(2-d), mass like n^(-d) relative to the n = 1 tables
double sA(hhg_ctx c, int l) { return c->dim == 2 ? 1.0 : std::ldexp(1.0, -l); }
double sM(hhg_ctx c, int l) { return std::ldexp(1.0, -c->dim * l); }
bool p1(hhg_ctx c) { return c->opt.coefficient == HHG_KAPPA_P1; }
double omega(hhg_ctx c) { return c->opt.jacobi_omega > 0 ? c->opt.jacobi_omega : 2.0 / 3.0; }

hhg_status check_ready(hhg_ctx c) {
  if (!c) return HHG_EINVAL;
  if (!c->bound) { c->err = "no workspace bound"; return HHG_ESTATE; }
  if (p1(c) && !c->kappa_nodal_set) { c->err = "HHG_KAPPA_P1 needs hhg_set_kappa_nodal first"; return HHG_ESTATE; }
  return HHG_OK;
}

// ---------------------------------------------------------------------------------------
// precision-specific level arrays
template <typename T> struct Arr;
template <> struct Arr<double> {
  static double*& x(Level& l) { return l.x; }
  static double*& x2(Level& l) { return l.x2; }
  static double*& t(Level& l) { return l.t; }
  static double*& rc(Level& l) { return l.rc; }
};
template <> struct Arr<float> {
  static float*& x(Level& l) { return l.x32; }
  static float*& x2(Level& l) { return l.x2_32; }
  static float*& t(Level& l) { return l.t32; }
  static float*& rc(Level& l) { return l.b32; }
};

// interior smoother launch(es); while profiling, finest-level launches are bracketed by events
template <typename T>
void interior_launch(hhg_ctx c, int l, const LK& k, const T* x, T* y, const T* b, int col, int rb, int jac,
                     const T* pro_ec = nullptr, T* pro_t = nullptr, bool zero_start = false) {
  Level& lv = c->lev[l];
  const bool fine = l == c->L;
  const bool rec = fine && c->prof_on && c->prof_used + 2 <= (int)c->prof_ev.size();
  if (rec) (void)hipEventRecord((hipEvent_t)c->prof_ev[c->prof_used], ST(c));
  int64_t npts;
  if (col < 0) {   // all interior colours fused in one launch
    launch_gs_fused<T>(c->dim, p1(c), k, c->tab, const_cast<T*>(x), y, b, lv.d_tiles, (int)lv.tiles.size(), lv.d_itab,
                       lv.d_itab_off, rb, sA(c, l), fine, ST(c), pro_ec, pro_ec ? (int)c->lev[l - 1].S : 0, pro_t,
                       zero_start);
    npts = lv.NI * c->nC;
  } else {
    launch_smooth_interior<T>(c->dim, p1(c), k, c->tab, x, y, b, col, rb, jac, omega(c), sA(c, l), lv.kn, fine, ST(c));
    npts = jac ? lv.NI * c->nC : lv.interior_per_colour[col];
  }
  if (rec) {
    (void)hipEventRecord((hipEvent_t)c->prof_ev[c->prof_used + 1], ST(c));
    c->prof_used += 2;
    const double per = (double)sizeof(T) * 3.0 + (p1(c) ? 8.0 : 0.0);
    c->prof_bytes += per * (double)npts;
  }
}

bool fused_available(hhg_ctx c, int l, size_t tsize) {
  const Level& lv = c->lev[l];
  if (p1(c) || lv.NI <= 0 || c->opt.smoother == HHG_JACOBI || c->no_fused) return false;
  if (c->dim == 2) return !lv.tiles.empty();
  // the whole-plane 3D sweep serves float32 only: in float64 (twice the LDS per plane, one
  // workgroup per compute unit) the class-by-class sweep measured faster
  if (lv.planes3d) return tsize == 4;
  if (!lv.tiles.empty()) return true;   // the plane-streaming 3D sweep
  return !lv.itab.empty() && (size_t)lv.Sraw * tsize <= 64 * 1024;
}

// the cycle's prolongation x_l += P e_{l-1} can run inside the first post-smoothing sweep, and
// a sweep on a zero iterate can start without reading (or clearing) it (2D fused out-of-place
// sweep, float32: in float64 the longer sweep measured slower than the two launches)
bool pro_fusable(hhg_ctx c, int l, size_t tsize) {
  return c->dim == 2 && tsize == 4 && l >= 1 && !c->no_pro && fused_available(c, l, tsize);
}

// sweeps of the level-l smoother.  With pro (pro_fusable), the first sweep starts from
// x_l + P pro; with zero_start (pro_fusable), from x_l = 0 whatever x_l holds.  Its interior
// launch forms that start on load and writes the start values of the macro-boundary nodes to
// t_l, from which the interface classes of that sweep read.
template <typename T>
hhg_status smooth(hhg_ctx c, int l, const T* b, int sweeps, const T* pro = nullptr, bool zero_start = false) {
  Level& lv = c->lev[l];
  const LK k = lk_of(c, l);
  const bool jac = c->opt.smoother == HHG_JACOBI;
  const int rb = c->opt.smoother == HHG_GS_REDBLACK ? 1 : 0;
  const bool fused = fused_available(c, l, sizeof(T));
  // out-of-place interior sweep (k_gs2d_fused, k_gs3d_planes, k_gs3d_stream)
  const bool twobuf = fused && (c->dim == 2 || !lv.tiles.empty());
  if (!jac && lv.NI == 0 && lv.task_ok && !c->no_tasks && !lv.fused_iface && sweeps > 1) {
    // no macro interiors (n = 2) and every interface class in the single-workgroup form that
    // does not preload: all sweeps in one launch, the same class sequence repeated
    bool one = true, pre = !c->no_preload;
    for (int cc = lv.interior_colours; cc < lv.ncolours; ++cc) {
      const int wv = lv.task_woff[cc + 1] - lv.task_woff[cc];
      if (wv > kTaskOneGroupWaves) one = false;
      if (wv > 16) pre = false;
    }
    if (pre && lv.ncolours - lv.interior_colours <= iface_pre_classes(c->dim, sizeof(T) == 8)) one = false;
    if (one) {
      T* x = Arr<T>::x(lv);
      launch_iface_tasks_1wg<T>(c->dim, k, c->tab, lv.d_task_copy, lv.d_task_info, lv.d_task_loc, lv.d_task_seg,
                                lv.d_task_wmax, lv.d_task_woff, lv.interior_colours, lv.ncolours, x, x, x, (T*)nullptr,
                                b, sA(c, l), false, ST(c), sweeps);
      LAUNCHCHK();
      return HHG_OK;
    }
  }
  for (int s = 0; s < sweeps; ++s) {
    T* x = Arr<T>::x(lv);
    if (jac) {
      T* y = Arr<T>::t(lv);
      interior_launch<T>(c, l, k, x, y, b, 0, 0, 1);
      launch_smooth_iface<T>(c->dim, p1(c), k, c->tab, nullptr, (int)lv.nIface, x, x, y, (T*)nullptr, b, 1, omega(c),
                             sA(c, l), lv.kn, ST(c));
      std::swap(Arr<T>::x(lv), Arr<T>::t(lv));
      c->xswap ^= 1u << (l + (sizeof(T) == 4 ? 16 : 0));
      continue;
    }
    // macro interiors first (all colours), then the interface colour classes; with two buffers
    // the interface reads interior neighbours from the new buffer y and interface values from x
    // (current), and writes both
    T* y = twobuf ? Arr<T>::x2(lv) : x;
    const bool first = s == 0 && twobuf && c->dim == 2;
    const T* pe = first ? pro : (const T*)nullptr;
    const bool z = first && !pro && zero_start;
    if (fused) interior_launch<T>(c, l, k, x, y, b, -1, rb, 0, pe, Arr<T>::t(lv), z);
    else
      for (int col = 0; col < lv.interior_colours; ++col) interior_launch<T>(c, l, k, x, x, b, col, rb, 0);
    // the whole-plane 3D sweep also copies the interface values into y, so the interface
    // classes then update y in place: one buffer, no mirror writes.  After a fused
    // prolongation the old interface values are those in t.
    const bool in_y = twobuf && lv.planes3d;
    T* xo = pe || z ? Arr<T>::t(lv) : x;
    T* xf = in_y ? y : xo;
    T* mir = twobuf && !in_y ? xo : (T*)nullptr;
    if (lv.task_ok && !c->no_tasks) {
      // 2D with large edge classes: both edge classes in one launch by edge chunks; then, as
      // for all classes otherwise, a class of more than kTaskOneGroupWaves wavefronts gets a
      // grid of its own and runs of smaller consecutive classes share one single-workgroup
      // launch
      int col = lv.interior_colours;
      if (lv.fused_iface && !c->classwise_iface && lv.wheels && lv.wh_merge && twobuf && !c->two_launch_iface) {
        // edge and vertex classes in one launch (the wheels recompute their edge-class
        // neighbours); x is only read, so the interface needs no mirror writes
        launch_iface2d_sweep<T>(k, c->tab, (const int32_t*)(c->ws + c->o_erec), (int)c->nE, lv.d_dvcopy,
                                (int)lv.dvcopy.size(), lv.d_whcopy, lv.d_whinfo, lv.d_whloc, lv.d_whseg, lv.d_whsrc,
                                lv.d_whcw, lv.d_whwmax, (int)lv.wh_wmax.size(), lv.ncolours - lv.c_vr0, lv.d_whe2,
                                lv.d_wha2i, lv.d_wha2w, y, xo, y, b, sA(c, l), ST(c));
        col = lv.ncolours;
      } else if (lv.fused_iface && !c->classwise_iface) {
        launch_iface2d_edges<T>(k, (const int32_t*)(c->ws + c->o_erec), (int)c->nE, lv.d_dvcopy, (int)lv.dvcopy.size(),
                                y, xo, y, mir, b, sA(c, l), ST(c));
        col = lv.c_vr0;
        if (lv.wheels) {
          launch_iface2d_wheels<T>(k, c->tab, lv.d_whcopy, lv.d_whinfo, lv.d_whloc, lv.d_whseg, lv.d_whsrc, lv.d_whcw,
                                   lv.d_whwmax, (int)lv.wh_wmax.size(), lv.ncolours - lv.c_vr0, y, xo, y, mir, b,
                                   sA(c, l), ST(c));
          col = lv.ncolours;
        }
      }
      while (col < lv.ncolours) {
        auto waves = [&](int cc) { return lv.task_woff[cc + 1] - lv.task_woff[cc]; };
        if (waves(col) > kTaskOneGroupWaves) {
          launch_iface_tasks<T>(c->dim, k, c->tab, lv.d_task_copy, lv.d_task_info, lv.d_task_loc, lv.d_task_seg,
                                lv.d_task_wmax, lv.task_woff[col], lv.task_woff[col + 1], y, xf, y, mir, b, 0, 0.0,
                                sA(c, l), ST(c));
          ++col;
          continue;
        }
        int c1 = col;
        bool pre = !c->no_preload;
        while (c1 < lv.ncolours && waves(c1) <= kTaskOneGroupWaves) {
          if (waves(c1) > 16) pre = false;
          ++c1;
        }
        launch_iface_tasks_1wg<T>(c->dim, k, c->tab, lv.d_task_copy, lv.d_task_info, lv.d_task_loc, lv.d_task_seg,
                                  lv.d_task_wmax, lv.d_task_woff, col, c1, y, xf, y, mir, b, sA(c, l), pre, ST(c));
        col = c1;
      }
    } else if (lv.max_iface_class <= kIfaceOneGroup) {
      launch_iface_sweep_1wg<T>(c->dim, p1(c), k, c->tab, lv.d_colour_list, lv.d_colour_off, lv.interior_colours,
                                lv.ncolours, y, xf, y, mir, b, sA(c, l), lv.kn, ST(c));
    } else {
      for (int col = lv.interior_colours; col < lv.ncolours; ++col) {
        const int cnt = lv.colour_off[col + 1] - lv.colour_off[col];
        launch_smooth_iface<T>(c->dim, p1(c), k, c->tab, lv.d_colour_list + lv.colour_off[col], cnt, y, xf, y, mir, b, 0,
                               0.0, sA(c, l), lv.kn, ST(c));
      }
    }
    if (twobuf) {
      std::swap(Arr<T>::x(lv), Arr<T>::x2(lv));
      c->xswap ^= 1u << (l + (sizeof(T) == 4 ? 16 : 0));
    }
  }
  LAUNCHCHK();
  return HHG_OK;
}

// level-0 step: x (+)= A_II^{-1} r on the inner coarse vertices
template <typename T>
hhg_status coarse_step(hhg_ctx c, const T* b, bool x_is_zero) {
  Level& l0 = c->lev[0];
  T* x = Arr<T>::x(l0);
  auto solve = [&](const T* rhs, int acc) {
    if (c->coarse_factored)
      launch_coarse_factored<T>(c->n0, c->d_ccopy_off, c->d_ccopy, c->d_cperm, c->d_ainv, c->d_cscr, rhs, x, acc, ST(c));
    else
      launch_coarse<T>(c->n0, c->d_ccopy_off, c->d_ccopy, c->d_ainv, rhs, x, acc, ST(c));
  };
  if (x_is_zero) {
    solve(b, 0);
  } else {
    T* r = Arr<T>::t(l0);
    launch_apply<T, T>(c->dim, p1(c), lk_of(c, 0), c->tab, x, b, r, 0, sA(c, 0), 1.0, -1.0, 1, l0.kn, ST(c));
    solve(r, 1);
  }
  LAUNCHCHK();
  return HHG_OK;
}

template <typename T> constexpr int prec_of() { return sizeof(T) == 4 ? 1 : 0; }
template <typename T> T* dense_of(hhg_ctx c);
template <> double* dense_of<double>(hhg_ctx c) { return c->d_dense64; }
template <> float* dense_of<float>(hhg_ctx c) { return c->d_dense32; }
int64_t dense_key(int pre, int post) { return (int64_t)pre | ((int64_t)post << 16); }

// V(pre,post) cycle on level l for A x_l = b; x_is_zero lets the coarsest step skip a residual.
// On the dense-map level, a cycle from a zero iterate is one product with the map built for
// these sweep counts (the same linear map as the launches below, up to rounding).  zero_first:
// x_l has not been cleared, the first sweep starts from zero (pro_fusable levels only)
template <typename T>
hhg_status vcycle(hhg_ctx c, int l, const T* b, int pre, int post, bool x_is_zero, bool zero_first = false) {
  if (x_is_zero && l == c->dense_k && !c->dense_building && c->dense_key[prec_of<T>()] == dense_key(pre, post)) {
    const Level& lv = c->lev[l];
    launch_dense_map<T>(c->dense_rows, c->dense_ld, c->dense_kmax, c->d_dgat, (T*)c->d_dsum, dense_of<T>(c), b,
                        lv.nfull, c->d_doff, c->d_dcopy, Arr<T>::x(c->lev[l]), ST(c));
    LAUNCHCHK();
    return HHG_OK;
  }
  if (l == 0) return coarse_step<T>(c, b, x_is_zero);
  Level& lv = c->lev[l];
  Level& lc = c->lev[l - 1];
  TRY(smooth<T>(c, l, b, pre, nullptr, zero_first));
  launch_apply<T, T>(c->dim, p1(c), lk_of(c, l), c->tab, Arr<T>::x(lv), b, Arr<T>::t(lv), 0, sA(c, l), 1.0, -1.0, 1,
                     lv.kn, ST(c));
  // restriction; the same launch clears the coarse correction (homogeneous, Dirichlet copies included)
  launch_restrict<T>(c->dim, lk_of(c, l), lk_of(c, l - 1), c->tab, Arr<T>::t(lv), Arr<T>::rc(lc), ST(c), Arr<T>::x(lc));
  TRY(vcycle<T>(c, l - 1, Arr<T>::rc(lc), pre, post, true));
  if (post >= 1 && pro_fusable(c, l, sizeof(T))) {
    TRY(smooth<T>(c, l, b, post, Arr<T>::x(lc)));
  } else {
    launch_prolong<T>(c->dim, lk_of(c, l), lk_of(c, l - 1), c->tab, Arr<T>::x(lc), Arr<T>::x(lv), (T*)nullptr,
                      (const T*)nullptr, 0, ST(c));
    TRY(smooth<T>(c, l, b, post));
  }
  LAUNCHCHK();
  return HHG_OK;
}

// Build the dense map of level dense_k for this precision and these sweep counts, unless it
// is there: one probe per inner DoF r (b_k = 1 at one copy of r, x_k = 0, the cycle of levels
// k .. 0 by its ordinary launches), whose result is column r of the map.  The cycle reads b_k
// only through the sums of each DoF's dual copies, so the map acts on those sums.  Runs
// eagerly, outside any recording, before a solve touches the level vectors.
template <typename T>
hhg_status ensure_dense_t(hhg_ctx c, int pre, int post) {
  const int k = c->dense_k;
  const int64_t key = dense_key(pre, post);
  if (k < 1 || c->dense_key[prec_of<T>()] == key) return HHG_OK;
  Level& lv = c->lev[k];
  T* B = dense_of<T>(c);
  c->dense_key[prec_of<T>()] = -1;
  launch_fill<T>(B, (int64_t)c->dense_rows * c->dense_ld, (T)0, ST(c));
  c->dense_building = true;
  for (int r = 0; r < c->dense_rows; ++r) {
    T* rc = Arr<T>::rc(lv);
    launch_unit<T>(rc, lv.nfull, c->dense_copy[c->dense_off[r]], ST(c));
    launch_fill<T>(Arr<T>::x(lv), lv.nfull, (T)0, ST(c));
    const hhg_status s = vcycle<T>(c, k, rc, pre, post, true);
    if (s != HHG_OK) { c->dense_building = false; return s; }
    launch_dense_harvest<T>(c->dense_rows, c->d_doff, c->d_dcopy, c->dense_ld, r, Arr<T>::x(lv), B, ST(c));
  }
  c->dense_building = false;
  LAUNCHCHK();
  c->dense_key[prec_of<T>()] = key;
  return HHG_OK;
}

hhg_status ensure_dense(hhg_ctx c, const hhg_solve_params& p) {
  return p.precision == HHG_FP64 ? ensure_dense_t<double>(c, p.pre, p.post) : ensure_dense_t<float>(c, p.pre, p.post);
}

// float64 residual of level l rounded to the float32 right-hand side b32_l of the correction
// equation; interface rows are summed over their copies in float64 before rounding and kept
// in the owner copy only
void residual_f32(hhg_ctx c, int l, const double* b) {
  Level& lv = c->lev[l];
  launch_apply<double, float>(c->dim, p1(c), lk_of(c, l), c->tab, lv.x, b, lv.b32, 0, sA(c, l), 1.0, -1.0, 1, lv.kn,
                              ST(c));
  // by lanes in 2D (two or a few copies per DoF); in 3D, where edge and vertex DoFs have many
  // copies, the one-thread-per-DoF kernel measured faster
  if (c->dim == 2 && lv.task_ok && !c->no_tasks)
    launch_iface_residual_tasks<double, float>(c->dim, lk_of(c, l), c->tab, lv.d_task_copy, lv.d_task_info,
                                               lv.d_task_loc, lv.d_task_seg, lv.d_task_wmax,
                                               lv.task_woff[lv.interior_colours], lv.task_woff[lv.ncolours], lv.x, b,
                                               lv.b32, sA(c, l), ST(c));
  else
    launch_iface_residual<double, float>(c->dim, p1(c), lk_of(c, l), c->tab, lv.x, b, lv.b32, sA(c, l), lv.kn, ST(c));
}

// one cycle on level l of the selected precision for x_l (float64) and rhs bf_l; with
// rhs_ready the float32 right-hand side b32_l already holds the current residual
hhg_status cycle(hhg_ctx c, int l, const double* b, const hhg_solve_params& p, bool rhs_ready = false) {
  Level& lv = c->lev[l];
  if (p.precision == HHG_FP64) return vcycle<double>(c, l, b, p.pre, p.post, false);
  if (!rhs_ready) residual_f32(c, l, b);
  // the correction starts from zero; the first sweep can start from zero without the clear
  // (not on the dense-map level, whose product writes the inner DoFs only)
  const bool zs = l >= 1 && l != c->dense_k && p.pre >= 1 && pro_fusable(c, l, sizeof(float));
  if (!zs) launch_fill<float>(lv.x32, lv.nfull, 0.0f, ST(c));
  TRY(vcycle<float>(c, l, lv.b32, p.pre, p.post, l == 0 || zs, zs));
  launch_add_f32(lv.x, lv.x32, lv.nfull, ST(c));
  LAUNCHCHK();
  return HHG_OK;
}

// ||b - A x|| over the non-Dirichlet DoFs of level l (uses t_l), returned on the host
hhg_status residual_norm(hhg_ctx c, int l, const double* x, const double* b, double* out) {
  Level& lv = c->lev[l];
  launch_apply<double, double>(c->dim, p1(c), lk_of(c, l), c->tab, x, b, lv.t, 0, sA(c, l), 1.0, -1.0, 1, lv.kn, ST(c));
  launch_sqnorm(c->dim, lk_of(c, l), c->tab, lv.t, c->d_red, c->d_scal, ST(c));
  LAUNCHCHK();
  double h = 0;
  HIPCHK(hipMemcpyAsync(&h, c->d_scal, sizeof(double), hipMemcpyDeviceToHost, ST(c)));
  HIPCHK(hipStreamSynchronize(ST(c)));
  *out = std::sqrt(h);
  return HHG_OK;
}

void drop_graphs(hhg_ctx c) {
  for (auto& g : c->graphs) (void)hipGraphExecDestroy((hipGraphExec_t)g.exec);
  c->graphs.clear();
}

// Run body() on the caller's stream, through a recorded HIP graph when possible: the first
// call with a key records body() on the private capture stream (nothing executes while
// recording), later calls replay it.  body() must only launch kernels (no copies, no
// synchronisation) and must leave the host-side buffer roles as it found them; the callers
// guarantee the latter by using graphs only for even pre- and post-smoothing counts (each
// out-of-place sweep swaps the two iterate buffers).
template <class F>
hhg_status run_recorded(hhg_ctx c, int64_t key, F&& body, int64_t key2 = 0) {
  // no graphs with the static workspace: instantiating one allocates
  if (c->no_graph || c->static_ws || c->prof_on || c->capturing) return body();
  hipGraphExec_t ex = nullptr;
  for (auto& g : c->graphs)
    if (g.key == key && g.key2 == key2) ex = (hipGraphExec_t)g.exec;
  if (!ex) {
    if (!c->cap_stream) {
      hipStream_t cs;
      HIPCHK(hipStreamCreate(&cs));
      c->cap_stream = cs;
    }
    HIPCHK(hipStreamBeginCapture((hipStream_t)c->cap_stream, hipStreamCaptureModeThreadLocal));
    c->capturing = true;
    const hhg_status s = body();
    c->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture((hipStream_t)c->cap_stream, &g);
    if (s != HHG_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess || !g) { c->err = std::string("HIP graph capture: ") + hipGetErrorString(e); return HHG_EHIP; }
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) { c->err = std::string("HIP graph instantiation: ") + hipGetErrorString(ei); return HHG_EHIP; }
    c->graphs.push_back({key, key2, (void*)ex});
  }
  HIPCHK(hipGraphLaunch(ex, (hipStream_t)c->stream));
  return HHG_OK;
}

// recorded launches refer to the iterate buffers by address, so the key includes which buffer
// of each level currently holds the iterate (an odd number of sweeps through hhg_smooth or
// hhg_bench_smoother leaves them exchanged)
int64_t graph_key(hhg_ctx c, int kind, const hhg_solve_params& p) {
  return (int64_t)kind | ((int64_t)p.nu << 4) | ((int64_t)p.pre << 12) | ((int64_t)p.post << 20) |
         ((int64_t)p.precision << 28) | ((int64_t)c->xswap << 32);
}

// FMG given bf_l and g_l on all levels; result in lev[L].x, w_l in lev[l+1].w
hhg_status fmg_core(hhg_ctx c, const hhg_solve_params& p, hhg_solve_stats* stats, bool warm = false) {
  const int L = c->L;
  const bool rec = p.pre % 2 == 0 && p.post % 2 == 0;
  auto body = [&]() -> hhg_status {
    Level& l0 = c->lev[0];
    launch_init_dirichlet(c->dim, lk_of(c, 0), c->tab, l0.g, l0.x, 0.0, ST(c));
    TRY(coarse_step<double>(c, l0.bf, false));
    for (int l = 1; l <= L; ++l) {
      Level& lv = c->lev[l];
      launch_prolong<double>(c->dim, lk_of(c, l), lk_of(c, l - 1), c->tab, c->lev[l - 1].x, lv.x, lv.w, lv.g, 2, ST(c));
      for (int it = 0; it < p.nu; ++it) TRY(cycle(c, l, lv.bf, p));
    }
    LAUNCHCHK();
    return HHG_OK;
  };
  // warm: the iterate on level L is given; only the cycles below run
  int vcycles = warm ? 0 : p.nu * L;
  if (p.max_iter > 0 && p.rtol == 0.0) {
    // a fixed number of extra cycles, no residual norms: the FMG pass and the cycles are one
    // launch sequence (one recorded graph)
    Level& lL = c->lev[L];
    auto all = [&]() -> hhg_status {
      if (!warm) TRY(body());
      for (int it = 0; it < p.max_iter; ++it) TRY(cycle(c, L, lL.bf, p));
      return HHG_OK;
    };
    TRY(rec ? run_recorded(c, graph_key(c, 4, p), all, (int64_t)p.max_iter | ((int64_t)warm << 32)) : all());
    if (stats) {
      stats->vcycles = vcycles + p.max_iter;
      stats->ir_steps = p.max_iter;
      stats->final_rel_residual = -1.0;
    }
    c->res_hist.clear();
    return HHG_OK;
  }
  if (!warm) TRY(rec ? run_recorded(c, graph_key(c, 1, p), body) : body());
  int extra = 0;
  double rel = -1.0;   // not computed without extra cycles
  if (p.max_iter > 0) {
    Level& lL = c->lev[L];
    // reference residual: u = g on the boundary, 0 inside (assembled into rc_L as scratch)
    launch_init_dirichlet(c->dim, lk_of(c, L), c->tab, lL.g, c->d_aux1, 0.0, ST(c));
    double r0 = 0, r = 0;
    TRY(residual_norm(c, L, c->d_aux1, lL.bf, &r0));
    TRY(residual_norm(c, L, lL.x, lL.bf, &r));
    rel = r0 > 0 ? r / r0 : 0.0;
    c->res_hist.clear();
    while (extra < p.max_iter && rel > p.rtol) {
      // one cycle and the residual it leaves, then the norm to the host.  In the float32-refined
      // form the residual is the rounded, interface-assembled right-hand side of the next
      // cycle's correction equation (its norm is exact to float32 rounding of the entries),
      // so the next cycle does not recompute it
      const bool f32 = p.precision == HHG_FP32_REFINED, ready = f32 && extra > 0;
      auto step = [&]() -> hhg_status {
        TRY(cycle(c, L, lL.bf, p, ready));
        if (f32) {
          residual_f32(c, L, lL.bf);
          launch_sqnorm_closure<float>(c->dim, lk_of(c, L), lL.b32, c->d_red, c->d_scal, ST(c));
        } else {
          launch_apply<double, double>(c->dim, p1(c), lk_of(c, L), c->tab, lL.x, lL.bf, lL.t, 0, sA(c, L), 1.0, -1.0, 1,
                                       lL.kn, ST(c));
          launch_sqnorm(c->dim, lk_of(c, L), c->tab, lL.t, c->d_red, c->d_scal, ST(c));
        }
        LAUNCHCHK();
        return HHG_OK;
      };
      TRY(rec ? run_recorded(c, graph_key(c, ready ? 3 : 2, p), step) : step());
      ++extra;
      ++vcycles;
      double h = 0;
      HIPCHK(hipMemcpyAsync(&h, c->d_scal, sizeof(double), hipMemcpyDeviceToHost, ST(c)));
      HIPCHK(hipStreamSynchronize(ST(c)));
      r = std::sqrt(h);
      rel = r0 > 0 ? r / r0 : 0.0;
      c->res_hist.push_back(rel);
      if (!std::isfinite(rel)) { c->err = "residual is not finite"; return HHG_ENOTCONV; }
      // stagnation: less than 10% reduction over the last four cycles
      const size_t nh = c->res_hist.size();
      if (nh >= 8 && rel > 0.9 * c->res_hist[nh - 5] && rel > p.rtol) {
        if (rel <= 1e-9) break;   // round-off floor of the float64 residual
        c->err = "extra cycles stagnate at relative residual " + std::to_string(rel) + " after " + std::to_string(extra) +
                 " cycles";
        if (stats) { stats->vcycles = vcycles; stats->ir_steps = extra; stats->final_rel_residual = rel; }
        return HHG_ENOTCONV;
      }
    }
  }
  if (stats) {
    stats->vcycles = vcycles;
    stats->ir_steps = extra;
    stats->final_rel_residual = rel;
  }
  return HHG_OK;
}

int dense_level_used(hhg_ctx c, const hhg_solve_params& p) {
  const int prec = p.precision == HHG_FP64 ? 0 : 1;
  return c->dense_k >= 1 && c->dense_key[prec] == dense_key(p.pre, p.post) ? c->dense_k : -1;
}

// right-hand sides of the primal problem on every level from nodal f and g on level L
hhg_status setup_rhs(hhg_ctx c, const double* f_nodal, const double* g_nodal) {
  const int L = c->L;
  Level& lL = c->lev[L];
  launch_canon_to_full(c->dim, lk_of(c, L), c->tab, f_nodal, lL.t, 0, ST(c));
  launch_canon_to_full(c->dim, lk_of(c, L), c->tab, g_nodal, lL.g, 0, ST(c));
  for (int l = 0; l < L; ++l) {
    launch_inject(c->dim, lk_of(c, L), lk_of(c, l), lL.t, c->lev[l].t, ST(c));
    launch_inject(c->dim, lk_of(c, L), lk_of(c, l), lL.g, c->lev[l].g, ST(c));
  }
  for (int l = 0; l <= L; ++l) {
    Level& lv = c->lev[l];
    launch_apply<double, double>(c->dim, false, lk_of(c, l), c->tab, lv.t, nullptr, lv.bf, 1, sM(c, l), 0.0, 1.0, 1,
                                 nullptr, ST(c));
  }
  LAUNCHCHK();
  return HHG_OK;
}

hhg_status validate_params(hhg_ctx c, const hhg_solve_params* p) {
  if (!p) { c->err = "params is NULL"; return HHG_EINVAL; }
  if (p->nu < 1 || p->pre < 0 || p->post < 0 || p->max_iter < 0 ||
      (p->precision != HHG_FP64 && p->precision != HHG_FP32_REFINED)) {
    c->err = "invalid solve parameters";
    return HHG_EINVAL;
  }
  return HHG_OK;
}

hhg_status upload_coarse(hhg_ctx c) {
  if (c->n0 > 0) {
    HIPCHK(hipMemcpyAsync(c->d_ainv, c->Ainv.data(), c->Ainv.size() * 8, hipMemcpyHostToDevice, ST(c)));
    HIPCHK(hipMemcpyAsync(c->d_cperm, c->coarse_perm.data(), c->coarse_perm.size() * 4, hipMemcpyHostToDevice,
                          ST(c)));
  }
  HIPCHK(hipStreamSynchronize(ST(c)));
  return HHG_OK;
}

// prolongate a level-`from` vector up to level `to` through the given per-level scratch
const double* prolong_chain(hhg_ctx c, const double* v, int from, int to, bool use_rc) {
  for (int l = from + 1; l <= to; ++l) {
    double* dst = use_rc ? c->lev[l].rc : c->lev[l].t;
    launch_prolong<double>(c->dim, lk_of(c, l), lk_of(c, l - 1), c->tab, v, dst, (double*)nullptr,
                           (const double*)nullptr, 1, ST(c));
    v = dst;
  }
  return v;
}

// per-macro [||u - a||_T^2, ||u - P b||_T^2] in the given norm into host vectors (u: level-L
// closure vector, the last solve's u_L unless given)
hhg_status estimate_pair(hhg_ctx c, int norm, const double* a, const double* bc, std::vector<double>& s1,
                         std::vector<double>& s2, const double* u = nullptr) {
  const int L = c->L;
  double* out = c->d_red + (c->red_capacity - 2 * c->nC - 8);
  launch_estimate(c->dim, norm, lk_of(c, L), lk_of(c, L - 1), c->tab, u ? u : c->lev[L].x, a, bc, c->d_red, out,
                  norm == HHG_NORM_ENERGY ? sA(c, L) : sM(c, L), !c->generic_est, ST(c));
  LAUNCHCHK();
  std::vector<double> h(2 * c->nC);
  HIPCHK(hipMemcpyAsync(h.data(), out, h.size() * 8, hipMemcpyDeviceToHost, ST(c)));
  HIPCHK(hipStreamSynchronize(ST(c)));
  s1.resize(c->nC);
  s2.resize(c->nC);
  for (int64_t m = 0; m < c->nC; ++m) { s1[m] = h[2 * m]; s2[m] = h[2 * m + 1]; }
  return HHG_OK;
}

// the pair of timing events of the solve entry points (not created for the static workspace)
hhg_status ensure_events(hhg_ctx c) {
  if (c->ev0) return HHG_OK;
  hipEvent_t a, b;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  c->ev0 = a;
  c->ev1 = b;
  return HHG_OK;
}

// record a timing event if the context has them
hipError_t record(hhg_ctx c, void* ev) { return ev ? hipEventRecord((hipEvent_t)ev, ST(c)) : hipSuccess; }

// milliseconds between the two timing events (0 without events)
hhg_status elapsed(hhg_ctx c, double* ms) {
  *ms = 0.0;
  if (!c->ev0) return HHG_OK;
  HIPCHK(hipEventSynchronize((hipEvent_t)c->ev1));
  float t = 0;
  HIPCHK(hipEventElapsedTime(&t, (hipEvent_t)c->ev0, (hipEvent_t)c->ev1));
  *ms = t;
  return HHG_OK;
}

// bind a workspace: clear it, upload the tables, point the level arrays into it.  With
// no_alloc (the static workspace) the clear is a fill kernel and no HIP events are created.
hhg_status bind_impl(hhg_ctx c, void* ptr, void* stream, bool no_alloc) {
  // recorded launches of a previous binding may still run on the old stream
  if (c->bound) HIPCHK(hipStreamSynchronize(ST(c)));
  drop_graphs(c);
  c->bound = false;
  c->ws = (char*)ptr;
  c->stream = stream;
  hipStream_t st = ST(c);
  const int d = c->dim, nv = d + 1;
  char* w = c->ws;
  if (no_alloc) launch_fill<float>((float*)w, (int64_t)(c->ws_bytes / 4), 0.0f, st);
  else HIPCHK(hipMemsetAsync(w, 0, c->ws_bytes, st));
  auto up = [&](int64_t off, const void* src, size_t n) -> hipError_t {
    if (n == 0) return hipSuccess;
    return hipMemcpyAsync(w + off, src, n, hipMemcpyHostToDevice, st);
  };
  fill_kappa_tables(c);
  HIPCHK(up(c->o_erec, c->erec.data(), c->erec.size() * 4));
  HIPCHK(up(c->o_stiff, c->stiff.data(), c->stiff.size() * 8));
  HIPCHK(up(c->o_mass, c->mass.data(), c->mass.size() * 8));
  HIPCHK(up(c->o_elemK, c->elemK.data(), c->elemK.size() * 8));
  HIPCHK(up(c->o_kappa, c->kappa_cell.data(), c->kappa_cell.size() * 8));
  HIPCHK(up(c->o_subprim, c->subprim.data(), c->subprim.size() * 4));
  HIPCHK(up(c->o_suborder, c->suborder.data(), c->suborder.size()));
  HIPCHK(up(c->o_dirbits, c->dirbits.data(), c->dirbits.size() * 2));
  HIPCHK(up(c->o_ownbits, c->ownbits.data(), c->ownbits.size() * 2));
  HIPCHK(up(c->o_rbpar, c->rbpar.data(), c->rbpar.size() * 4));
  HIPCHK(up(c->o_incoff, c->inc_off.data(), c->inc_off.size() * 4));
  HIPCHK(up(c->o_inc, c->inc.data(), c->inc.size() * sizeof(Inc)));
  HIPCHK(up(c->o_primdir, c->primdir.data(), c->primdir.size()));
  HIPCHK(up(c->o_ccopyoff, c->coarse_copy_off.data(), c->coarse_copy_off.size() * 4));
  HIPCHK(up(c->o_ccopy, c->coarse_copy.data(), c->coarse_copy.size() * 8));
  std::vector<double> mx(c->nC * nv * d);
  for (int64_t m = 0; m < c->nC; ++m)
    for (int a = 0; a < nv; ++a)
      for (int q = 0; q < d; ++q) mx[(m * nv + a) * d + q] = c->coords[c->cells[m * nv + a] * d + q];
  HIPCHK(up(c->o_mxyz, mx.data(), mx.size() * 8));
  Tables& t = c->tab;
  t.dim = d;
  t.nmacro = (int)c->nC;
  t.nV = (int)c->nV;
  t.nE = c->nE;
  t.nF = c->nF;
  t.stiff = (const double*)(w + c->o_stiff);
  t.mass = (const double*)(w + c->o_mass);
  t.elemK = (const double*)(w + c->o_elemK);
  t.kappa = (const double*)(w + c->o_kappa);
  t.subprim = (const int32_t*)(w + c->o_subprim);
  t.suborder = (const uint8_t*)(w + c->o_suborder);
  t.dirbits = (const uint16_t*)(w + c->o_dirbits);
  t.ownbits = (const uint16_t*)(w + c->o_ownbits);
  t.rbpar = (const int32_t*)(w + c->o_rbpar);
  t.inc_off = (const int32_t*)(w + c->o_incoff);
  t.inc = (const Inc*)(w + c->o_inc);
  t.primdir = (const uint8_t*)(w + c->o_primdir);
  for (int q = 0; q < kMaxMask; ++q) { t.validdirs[q] = c->validdirs[q]; t.incvalid[q] = c->incvalid[q]; }
  c->d_red = (double*)(w + c->o_red);
  c->d_scal = (double*)(w + c->o_scal);
  c->d_ccopy_off = (int32_t*)(w + c->o_ccopyoff);
  c->d_ccopy = (int64_t*)(w + c->o_ccopy);
  c->d_ainv = (double*)(w + c->o_ainv);
  c->d_cperm = (int32_t*)(w + c->o_cperm);
  c->d_cscr = (double*)(w + c->o_cscr);
  c->d_aux0 = (double*)(w + c->o_aux0);
  c->d_aux1 = (double*)(w + c->o_aux1);
  c->d_dense32 = (float*)(w + c->o_dense32);
  c->d_dense64 = (double*)(w + c->o_dense64);
  c->d_doff = (int32_t*)(w + c->o_doff);
  c->d_dcopy = (int32_t*)(w + c->o_dcopy);
  c->d_dgat = (int32_t*)(w + c->o_dgat);
  c->d_dsum = (void*)(w + c->o_dsum);
  HIPCHK(up(c->o_doff, c->dense_off.data(), c->dense_off.size() * 4));
  HIPCHK(up(c->o_dcopy, c->dense_copy.data(), c->dense_copy.size() * 4));
  HIPCHK(up(c->o_dgat, c->dense_gat.data(), c->dense_gat.size() * 4));
  c->dense_key[0] = c->dense_key[1] = -1;
  for (auto& lv : c->lev) {
    lv.x = (double*)(w + lv.off_x);
    lv.t = (double*)(w + lv.off_t);
    lv.bf = (double*)(w + lv.off_bf);
    lv.rc = (double*)(w + lv.off_rc);
    lv.g = (double*)(w + lv.off_g);
    lv.w = (double*)(w + lv.off_w);
    lv.kn = lv.off_kn >= 0 ? (double*)(w + lv.off_kn) : nullptr;
    lv.x32 = (float*)(w + lv.off_x32);
    lv.x2 = (double*)(w + lv.off_x2);
    lv.x2_32 = (float*)(w + lv.off_x2_32);
    lv.t32 = (float*)(w + lv.off_t32);
    lv.b32 = (float*)(w + lv.off_b32);
    lv.d_colour_list = (int32_t*)(w + lv.off_cl);
    HIPCHK(up(lv.off_cl, lv.colour_list.data(), lv.colour_list.size() * 4));
    lv.d_task_copy = (int32_t*)(w + lv.off_tcopy);
    HIPCHK(up(lv.off_tcopy, lv.task_copy.data(), lv.task_copy.size() * 4));
    lv.d_task_info = (int32_t*)(w + lv.off_tinfo);
    HIPCHK(up(lv.off_tinfo, lv.task_info.data(), lv.task_info.size() * 4));
    lv.d_task_loc = (int32_t*)(w + lv.off_tloc);
    HIPCHK(up(lv.off_tloc, lv.task_loc.data(), lv.task_loc.size() * 4));
    lv.d_task_seg = (int32_t*)(w + lv.off_tseg);
    HIPCHK(up(lv.off_tseg, lv.task_seg.data(), lv.task_seg.size() * 4));
    lv.d_task_wmax = (int32_t*)(w + lv.off_twmax);
    HIPCHK(up(lv.off_twmax, lv.task_wmax.data(), lv.task_wmax.size() * 4));
    lv.d_task_woff = (int32_t*)(w + lv.off_twoff);
    HIPCHK(up(lv.off_twoff, lv.task_woff.data(), lv.task_woff.size() * 4));
    lv.d_dvcopy = (int32_t*)(w + lv.off_dvcopy);
    HIPCHK(up(lv.off_dvcopy, lv.dvcopy.data(), lv.dvcopy.size() * 4));
    lv.d_whcopy = (int32_t*)(w + lv.off_whcopy);
    HIPCHK(up(lv.off_whcopy, lv.wh_copy.data(), lv.wh_copy.size() * 4));
    lv.d_whinfo = (int32_t*)(w + lv.off_whinfo);
    HIPCHK(up(lv.off_whinfo, lv.wh_info.data(), lv.wh_info.size() * 4));
    lv.d_whloc = (int32_t*)(w + lv.off_whloc);
    HIPCHK(up(lv.off_whloc, lv.wh_loc.data(), lv.wh_loc.size() * 4));
    lv.d_whseg = (int32_t*)(w + lv.off_whseg);
    HIPCHK(up(lv.off_whseg, lv.wh_seg.data(), lv.wh_seg.size() * 4));
    lv.d_whsrc = (int32_t*)(w + lv.off_whsrc);
    HIPCHK(up(lv.off_whsrc, lv.wh_src.data(), lv.wh_src.size() * 4));
    lv.d_whwmax = (int32_t*)(w + lv.off_whwmax);
    HIPCHK(up(lv.off_whwmax, lv.wh_wmax.data(), lv.wh_wmax.size() * 4));
    lv.d_whcw = (double*)(w + lv.off_whcw);
    HIPCHK(up(lv.off_whcw, lv.wh_cw.data(), lv.wh_cw.size() * 8));
    lv.d_whe2 = (int32_t*)(w + lv.off_whe2);
    HIPCHK(up(lv.off_whe2, lv.wh_e2.data(), lv.wh_e2.size() * 4));
    lv.d_wha2i = (int32_t*)(w + lv.off_wha2i);
    HIPCHK(up(lv.off_wha2i, lv.wh_a2i.data(), lv.wh_a2i.size() * 4));
    lv.d_wha2w = (double*)(w + lv.off_wha2w);
    HIPCHK(up(lv.off_wha2w, lv.wh_a2w.data(), lv.wh_a2w.size() * 8));
    lv.d_colour_off = (int32_t*)(w + lv.off_coff);
    HIPCHK(up(lv.off_coff, lv.colour_off.data(), lv.colour_off.size() * 4));
    lv.d_tiles = (int32_t*)(w + lv.off_tiles);
    HIPCHK(up(lv.off_tiles, lv.tiles.data(), lv.tiles.size() * 4));
    lv.d_itab = (uint32_t*)(w + lv.off_itab);
    HIPCHK(up(lv.off_itab, lv.itab.data(), lv.itab.size() * 4));
    lv.d_itab_off = (int32_t*)(w + lv.off_itoff);
    HIPCHK(up(lv.off_itoff, lv.itab_off.data(), lv.itab_off.size() * 4));
  }
  if (!no_alloc) TRY(ensure_events(c));
  c->bound = true;
  c->solved = false;
  c->have_u = false;
  return upload_coarse(c);
}


constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};      // device address of scratch per device (looked up once)
hhg_ctx g_static_owner[kMaxDevices] = {};  // the context bound to it per device

// release c's claim on a static workspace (rebinding, destruction)
void release_static(hhg_ctx c) {
  if (c->static_dev < 0) return;
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (g_static_owner[c->static_dev] == c) g_static_owner[c->static_dev] = nullptr;
  c->static_dev = -1;
}

}  // namespace

// The static workspace of hhg_bind_static_workspace: one array per device, found through
// hipGetSymbolAddress on first use on that device; host code uses only those addresses.
static __device__ __align__(256) unsigned char scratch[HHG_STATIC_WORKSPACE_BYTES];

// =========================================================================================
extern "C" {

const char* hhg_status_string(hhg_status s) {
  switch (s) {
    case HHG_OK: return "HHG_OK";
    case HHG_EINVAL: return "HHG_EINVAL: invalid argument";
    case HHG_EMESH: return "HHG_EMESH: invalid mesh";
    case HHG_ENOMEM: return "HHG_ENOMEM: workspace too small";
    case HHG_EHIP: return "HHG_EHIP: HIP runtime error";
    case HHG_ENOTCONV: return "HHG_ENOTCONV: no convergence";
    case HHG_ESTATE: return "HHG_ESTATE: wrong state";
  }
  return "unknown status";
}

const char* hhg_last_error(hhg_ctx c) { return c ? c->err.c_str() : g_err.c_str(); }

hhg_status hhg_setup(const hhg_mesh* mesh, int L, const hhg_options* opt, hhg_ctx* out) {
  if (!out) { g_err = "out is NULL"; return HHG_EINVAL; }
  *out = nullptr;
  if (!mesh || !opt) { g_err = "mesh or options is NULL"; return HHG_EINVAL; }
  if (mesh->dim != 2 && mesh->dim != 3) { g_err = "dim must be 2 or 3"; return HHG_EINVAL; }
  if (L < 1 || L > (mesh->dim == 3 ? 9 : 12)) { g_err = "level L out of range"; return HHG_EINVAL; }
  if (mesh->n_vertices <= 0 || mesh->n_cells <= 0 || !mesh->coords || !mesh->cells) { g_err = "empty mesh"; return HHG_EMESH; }
  if (opt->smoother < HHG_GS_REDBLACK || opt->smoother > HHG_JACOBI ||
      (opt->coefficient != HHG_KAPPA_MACRO && opt->coefficient != HHG_KAPPA_P1)) {
    g_err = "invalid options";
    return HHG_EINVAL;
  }
  // The nodal-coefficient path is switched off: a parity run of it ended in a GPU memory
  // fault whose cause was not found, so it is not offered until one is shown and fixed.
  if (opt->coefficient == HHG_KAPPA_P1) {
    g_err = "HHG_KAPPA_P1 (nodal coefficient) is switched off in this build";
    return HHG_EINVAL;
  }
  hhg_ctx c = new (std::nothrow) hhg_ctx_s();
  if (!c) { g_err = "out of host memory"; return HHG_ENOMEM; }
  c->dim = mesh->dim;
  c->L = L;
  c->opt = *opt;
  c->no_fused = (opt->flags & HHG_FLAG_NO_FUSED) != 0;
  c->no_tasks = (opt->flags & HHG_FLAG_NO_LANE_IFACE) != 0;
  c->classwise_iface = (opt->flags & HHG_FLAG_CLASSWISE_IFACE) != 0;
  c->no_graph = (opt->flags & HHG_FLAG_NO_GRAPH) != 0;
  c->no_preload = (opt->flags & HHG_FLAG_NO_PRELOAD) != 0;
  c->force_rows3d = (opt->flags & HHG_FLAG_ROWS3D) != 0;
  c->force_stream3d = (opt->flags & HHG_FLAG_STREAM3D) != 0;
  c->no_planes3d = (opt->flags & HHG_FLAG_NO_PLANES3D) != 0;
  c->force_planes3d = (opt->flags & HHG_FLAG_PLANES3D) != 0;
  c->two_launch_iface = (opt->flags & HHG_FLAG_TWO_LAUNCH_IFACE) != 0;
  c->generic_est = (opt->flags & HHG_FLAG_GENERIC_EST) != 0;
  c->no_dense = (opt->flags & HHG_FLAG_NO_DENSE_COARSE) != 0;
  c->force_dense = (opt->flags & HHG_FLAG_DENSE_COARSE) != 0;
  c->no_pro = (opt->flags & HHG_FLAG_NO_FUSED_PROLONG) != 0;
  c->nV = mesh->n_vertices;
  c->nC = mesh->n_cells;
  const int nv = c->dim + 1;
  c->coords.assign(mesh->coords, mesh->coords + c->nV * c->dim);
  c->cells.assign(mesh->cells, mesh->cells + c->nC * nv);
  c->kappa_cell.assign(c->nC, 1.0);
  if (mesh->kappa_cell) c->kappa_cell.assign(mesh->kappa_cell, mesh->kappa_cell + c->nC);
  for (double k : c->kappa_cell)
    if (!(k > 0) || !std::isfinite(k)) { g_err = "kappa_cell must be positive"; delete c; return HHG_EINVAL; }
  if (mesh->dirichlet) c->vdir_user.assign(mesh->dirichlet, mesh->dirichlet + c->nV);
  hhg_status s = build_topology(c);
  if (s == HHG_OK) s = build_stencils(c);
  if (s != HHG_OK) { g_err = c->err; delete c; return s; }
  // levels
  c->lev.resize(L + 1);
  for (int l = 0; l <= L; ++l) {
    Level& lv = c->lev[l];
    lv.l = l;
    lv.n = 1 << l;
    const int n = lv.n;
    lv.Sraw = c->dim == 3 ? tet_count(n) : tri_count(n);
    lv.S = (lv.Sraw + 63) / 64 * 64;
    lv.NI = c->dim == 3 ? tet_count(n - 4) : tri_count(n - 3);
    lv.nEd = n - 1;
    lv.nFd = tri_count(n - 3);
    lv.nIface = c->nV + (int64_t)c->nE * lv.nEd + (c->dim == 3 ? (int64_t)c->nF * lv.nFd : 0);
    lv.ndof = lv.nIface + c->nC * lv.NI;
    lv.nfull = c->nC * lv.S;
  }
  s = build_colouring(c);
  if (s == HHG_OK) s = build_coarse(c, nullptr);
  if (s != HHG_OK) { g_err = c->err; delete c; return s; }
  build_dense_plan(c);
  plan_workspace(c);
  *out = c;
  return HHG_OK;
}

hhg_status hhg_workspace_bytes(hhg_ctx c, size_t* bytes) {
  if (!c || !bytes) return HHG_EINVAL;
  *bytes = c->ws_bytes;
  return HHG_OK;
}

hhg_status hhg_bind_workspace(hhg_ctx c, void* ptr, size_t bytes, void* stream) {
  if (!c) return HHG_EINVAL;
  if (!ptr || bytes < c->ws_bytes) { c->err = "workspace too small"; return HHG_ENOMEM; }
  if (((uintptr_t)ptr & 255) != 0) { c->err = "workspace must be 256-byte aligned"; return HHG_EINVAL; }
  release_static(c);
  c->static_ws = false;
  return bind_impl(c, ptr, stream, false);
}

hhg_status hhg_bind_static_workspace(hhg_ctx c, void* stream) {
  if (!c) return HHG_EINVAL;
  if (c->ws_bytes > (size_t)HHG_STATIC_WORKSPACE_BYTES) {
    c->err = "the context needs " + std::to_string(c->ws_bytes) + " bytes of workspace, more than the " +
             std::to_string((size_t)HHG_STATIC_WORKSPACE_BYTES) + " bytes of the static workspace";
    return HHG_ENOMEM;
  }
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) { c->err = "device index beyond the static workspace table"; return HHG_EINVAL; }
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        c->err = std::string("hipGetSymbolAddress of the static workspace: ") + hipGetErrorString(e);
        return HHG_EHIP;
      }
      g_static_ptr[dev] = p;
    }
    ptr = g_static_ptr[dev];
    hhg_ctx prev = g_static_owner[dev];
    if (prev && prev != c) {
      // the previous owner's tables are about to be overwritten: it needs a new binding
      prev->bound = false;
      prev->solved = prev->have_u = false;
      prev->static_dev = -1;
    }
    if (c->static_dev >= 0 && c->static_dev != dev && g_static_owner[c->static_dev] == c)
      g_static_owner[c->static_dev] = nullptr;
    g_static_owner[dev] = c;
    c->static_dev = dev;
  }
  c->static_ws = true;
  const hhg_status s = bind_impl(c, ptr, stream, true);
  if (s != HHG_OK) release_static(c);
  return s;
}

hhg_status hhg_num_dofs(hhg_ctx c, int level, int64_t* n) {
  if (!c || !n) return HHG_EINVAL;
  if (level < 0 || level > c->L) { c->err = "level out of range"; return HHG_EINVAL; }
  *n = c->lev[level].ndof;
  return HHG_OK;
}

hhg_status hhg_dof_coords(hhg_ctx c, int level, double* xyz) {
  if (!c || !xyz) return HHG_EINVAL;
  if (!c->bound) { c->err = "no workspace bound"; return HHG_ESTATE; }
  if (level < 0 || level > c->L) { c->err = "level out of range"; return HHG_EINVAL; }
  launch_dof_coords(c->dim, lk_of(c, level), c->tab, (const double*)(c->ws + c->o_mxyz), nullptr, xyz, ST(c));
  LAUNCHCHK();
  return HHG_OK;
}

hhg_status hhg_set_kappa_cell(hhg_ctx c, const double* kappa) {
  if (!c || !kappa) return HHG_EINVAL;
  for (int64_t m = 0; m < c->nC; ++m)
    if (!(kappa[m] > 0) || !std::isfinite(kappa[m])) { c->err = "kappa_cell must be positive"; return HHG_EINVAL; }
  c->kappa_cell.assign(kappa, kappa + c->nC);
  c->dense_key[0] = c->dense_key[1] = -1;
  TRY(build_coarse(c, nullptr));
  fill_kappa_tables(c);
  if (c->bound) {
    HIPCHK(hipMemcpyAsync(c->ws + c->o_kappa, c->kappa_cell.data(), c->nC * 8, hipMemcpyHostToDevice, ST(c)));
    if (!c->erec.empty())
      HIPCHK(hipMemcpyAsync(c->ws + c->o_erec, c->erec.data(), c->erec.size() * 4, hipMemcpyHostToDevice, ST(c)));
    for (auto& lv : c->lev) {
      if (!lv.wh_cw.empty())
        HIPCHK(hipMemcpyAsync(c->ws + lv.off_whcw, lv.wh_cw.data(), lv.wh_cw.size() * 8, hipMemcpyHostToDevice, ST(c)));
      if (!lv.wh_a2w.empty())
        HIPCHK(hipMemcpyAsync(c->ws + lv.off_wha2w, lv.wh_a2w.data(), lv.wh_a2w.size() * 8, hipMemcpyHostToDevice,
                              ST(c)));
    }
    TRY(upload_coarse(c));
  }
  c->solved = false;
  c->have_u = false;
  return HHG_OK;
}

hhg_status hhg_set_kappa_nodal(hhg_ctx c, const double* kappa) {
  if (!c || !kappa) return HHG_EINVAL;
  if (!p1(c)) { c->err = "hhg_set_kappa_nodal needs HHG_KAPPA_P1"; return HHG_ESTATE; }
  if (!c->bound) { c->err = "no workspace bound"; return HHG_ESTATE; }
  const int L = c->L;
  launch_canon_to_full(c->dim, lk_of(c, L), c->tab, kappa, c->lev[L].kn, 0, ST(c));
  for (int l = 0; l < L; ++l) launch_inject(c->dim, lk_of(c, L), lk_of(c, l), c->lev[L].kn, c->lev[l].kn, ST(c));
  LAUNCHCHK();
  std::vector<double> kv(c->nV);
  HIPCHK(hipMemcpyAsync(kv.data(), kappa, c->nV * 8, hipMemcpyDeviceToHost, ST(c)));   // vertices lead the order
  HIPCHK(hipStreamSynchronize(ST(c)));
  for (double k : kv)
    if (!(k > 0) || !std::isfinite(k)) { c->err = "nodal kappa must be positive"; return HHG_EINVAL; }
  c->dense_key[0] = c->dense_key[1] = -1;
  TRY(build_coarse(c, kv.data()));
  TRY(upload_coarse(c));
  c->kappa_nodal_set = true;
  c->solved = false;
  c->have_u = false;
  return HHG_OK;
}

hhg_status hhg_fmg_solve(hhg_ctx c, const double* f, const double* g, double* u_out, const hhg_solve_params* p,
                         hhg_solve_stats* stats) {
  TRY(check_ready(c));
  TRY(validate_params(c, p));
  if (!f || !g || !u_out) { c->err = "NULL vector"; return HHG_EINVAL; }
  TRY(ensure_dense(c, *p));
  HIPCHK(record(c, c->ev0));
  TRY(setup_rhs(c, f, g));
  hhg_solve_stats st{};
  hhg_status s = fmg_core(c, *p, &st);
  if (s != HHG_OK && s != HHG_ENOTCONV) return s;
  launch_full_to_canon(c->dim, lk_of(c, c->L), c->tab, c->lev[c->L].x, u_out, 0, ST(c));
  LAUNCHCHK();
  HIPCHK(record(c, c->ev1));
  if (stats) {
    TRY(elapsed(c, &st.ms_total));
    st.dense_level = dense_level_used(c, *p);
    *stats = st;
  }
  c->solved = (s == HHG_OK);
  c->have_u = c->solved;
  c->last_nu = p->nu;
  return s;
}

hhg_status hhg_cycle_solve(hhg_ctx c, const double* f, const double* g, double* u, const hhg_solve_params* p,
                           hhg_solve_stats* stats) {
  TRY(check_ready(c));
  TRY(validate_params(c, p));
  if (!f || !g || !u) { c->err = "NULL vector"; return HHG_EINVAL; }
  if (p->max_iter < 1) { c->err = "hhg_cycle_solve needs max_iter >= 1"; return HHG_EINVAL; }
  c->solved = c->have_u = false;
  TRY(ensure_dense(c, *p));
  HIPCHK(record(c, c->ev0));
  TRY(setup_rhs(c, f, g));
  const int L = c->L;
  Level& lL = c->lev[L];
  launch_canon_to_full(c->dim, lk_of(c, L), c->tab, u, lL.x, 0, ST(c));
  launch_impose_dirichlet(c->dim, lk_of(c, L), c->tab, lL.g, lL.x, ST(c));
  LAUNCHCHK();
  hhg_solve_stats st{};
  hhg_status s = fmg_core(c, *p, &st, true);
  if (s != HHG_OK && s != HHG_ENOTCONV) return s;
  launch_full_to_canon(c->dim, lk_of(c, L), c->tab, lL.x, u, 0, ST(c));
  LAUNCHCHK();
  HIPCHK(record(c, c->ev1));
  if (stats) {
    TRY(elapsed(c, &st.ms_total));
    st.dense_level = dense_level_used(c, *p);
    *stats = st;
  }
  c->have_u = (s == HHG_OK);
  return s;
}

hhg_status hhg_transfer(hhg_ctx c, hhg_ctx old, const double* u_old, double* u_new) {
  TRY(check_ready(c));
  if (!old || !old->bound) { c->err = "the old context has no workspace bound"; return HHG_ESTATE; }
  if (c->dim != old->dim) { c->err = "the two meshes differ in dimension"; return HHG_EINVAL; }
  if (!u_old || !u_new) { c->err = "NULL vector"; return HHG_EINVAL; }
  const int d = c->dim, nv = d + 1;
  // candidate old macros of every new macro: those whose bounding boxes meet its own
  auto box = [d, nv](hhg_ctx k, int64_t m, double* b) {
    for (int q = 0; q < d; ++q) {
      b[2 * q] = 1e300;
      b[2 * q + 1] = -1e300;
    }
    for (int a = 0; a < nv; ++a) {
      const int v = k->cells[m * nv + a];
      for (int q = 0; q < d; ++q) {
        b[2 * q] = std::min(b[2 * q], k->coords[v * d + q]);
        b[2 * q + 1] = std::max(b[2 * q + 1], k->coords[v * d + q]);
      }
    }
  };
  std::vector<double> bo(old->nC * 6);
  double ext = 0.0;
  for (int64_t m = 0; m < old->nC; ++m) {
    box(old, m, &bo[m * 6]);
    for (int q = 0; q < d; ++q) ext = std::max(ext, bo[m * 6 + 2 * q + 1] - bo[m * 6 + 2 * q]);
  }
  const double tol = 1e-9 * ext;
  std::vector<int32_t> off(c->nC + 1, 0), cand;
  for (int64_t m = 0; m < c->nC; ++m) {
    double b[6];
    box(c, m, b);
    for (int64_t M = 0; M < old->nC; ++M) {
      const double* q = &bo[M * 6];
      bool meet = true;
      for (int a = 0; a < d; ++a) meet = meet && q[2 * a] <= b[2 * a + 1] + tol && b[2 * a] <= q[2 * a + 1] + tol;
      if (meet) cand.push_back((int32_t)M);
    }
    off[m + 1] = (int32_t)cand.size();
  }
  const int L = c->L;
  Level& ln = c->lev[L];
  Level& lo = old->lev[old->L];
  const size_t bytes = (off.size() + cand.size()) * sizeof(int32_t);
  if (bytes > (size_t)ln.nfull * sizeof(double)) { c->err = "too many candidate macros"; return HHG_EINVAL; }
  int32_t* d_off = reinterpret_cast<int32_t*>(c->d_aux1);
  int32_t* d_cand = d_off + off.size();
  HIPCHK(hipMemcpyAsync(d_off, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice, ST(c)));
  if (!cand.empty())
    HIPCHK(hipMemcpyAsync(d_cand, cand.data(), cand.size() * sizeof(int32_t), hipMemcpyHostToDevice, ST(c)));
  // the old vector into the old context's closure scratch, interpolated into the new one's
  launch_canon_to_full(d, lk_of(old, old->L), old->tab, u_old, lo.rc, 0, ST(c));
  launch_transfer(d, lk_of(c, L), (const double*)(c->ws + c->o_mxyz), lk_of(old, old->L),
                  (const double*)(old->ws + old->o_mxyz), d_off, d_cand, lo.rc, ln.t, ST(c));
  launch_full_to_canon(d, lk_of(c, L), c->tab, ln.t, u_new, 0, ST(c));
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(ST(c)));
  return HHG_OK;
}

hhg_status hhg_estimate_ex(hhg_ctx c, int j, int norm, int local, double* eta_cell, double* eta_j, double* theta_est,
                           double* norm_e) {
  TRY(check_ready(c));
  if (!c->solved) { c->err = "hhg_estimate needs a preceding successful hhg_fmg_solve"; return HHG_ESTATE; }
  const int L = c->L;
  if (j < 1 || j >= L) { c->err = "need 0 < j < L"; return HHG_EINVAL; }
  if (norm != HHG_NORM_L2 && norm != HHG_NORM_ENERGY && norm != HHG_NORM_LUMPED) {
    c->err = "unknown norm";
    return HHG_EINVAL;
  }
  if (local != HHG_LOCAL_L1 && local != HHG_LOCAL_UNSCALED && local != HHG_LOCAL_SCALED) {
    c->err = "unknown local indicator";
    return HHG_EINVAL;
  }
  if (norm == HHG_NORM_ENERGY && p1(c)) {
    c->err = "the energy norm is implemented for per-macro coefficients only";
    return HHG_EINVAL;
  }
  const int l = L - j;
  // w_k is stored on level k+1 (lev[k+1].w).  s_l[T] = ||e~_l||_T^2, s_lm1[T] = ||e~_{l-1}||_T^2.
  std::vector<double> s_l, s_lm1, a1;
  if (j == 1) {
    TRY(estimate_pair(c, norm, c->lev[L].w, c->lev[L - 1].w, s_l, s_lm1));
  } else {
    // e~_l = u_L - I_{l+1}^L w_l,  e~_{l-1} = u_L - I_l^L w_{l-1} (last prolongation fused)
    const double* A = prolong_chain(c, c->lev[l + 1].w, l + 1, L, true);
    const double* B = prolong_chain(c, c->lev[l].w, l, L - 1, false);
    TRY(estimate_pair(c, norm, A, B, s_l, s_lm1));
  }
  if (eta_cell && local == HHG_LOCAL_L1 && j > 1) {
    std::vector<double> unused;
    TRY(estimate_pair(c, norm, c->lev[L].w, c->lev[L - 1].w, a1, unused));
  }
  double n1 = 0, n2 = 0;
  for (int64_t m = 0; m < c->nC; ++m) { n1 += s_l[m]; n2 += s_lm1[m]; }
  n1 = std::sqrt(std::max(n1, 0.0));
  n2 = std::sqrt(std::max(n2, 0.0));
  const double theta = n2 > 0 ? n1 / n2 : 0.0;
  if (eta_cell) {
    for (int64_t m = 0; m < c->nC; ++m) {
      const double el = std::sqrt(std::max(s_l[m], 0.0));
      if (local == HHG_LOCAL_L1) {
        eta_cell[m] = std::sqrt(std::max(j == 1 ? s_l[m] : a1[m], 0.0));
      } else if (local == HHG_LOCAL_UNSCALED) {
        eta_cell[m] = el;
      } else {
        const double elm1 = std::sqrt(std::max(s_lm1[m], 0.0));
        eta_cell[m] = elm1 > 0 ? std::pow(el / elm1, j) * el : 0.0;
      }
    }
  }
  if (eta_j) *eta_j = std::pow(theta, j) * n1;
  if (theta_est) *theta_est = theta;
  if (norm_e) *norm_e = n1;
  return HHG_OK;
}

hhg_status hhg_macro_norms(hhg_ctx c, const double* x, int level, int norm, double* sq) {
  TRY(check_ready(c));
  const int L = c->L;
  if (!sq || level < -1 || level > L || (level == -1 && !x) ||
      (norm != HHG_NORM_L2 && norm != HHG_NORM_ENERGY && norm != HHG_NORM_LUMPED)) {
    c->err = "invalid argument";
    return HHG_EINVAL;
  }
  if (norm == HHG_NORM_ENERGY && p1(c)) {
    c->err = "the energy norm is implemented for per-macro coefficients only";
    return HHG_EINVAL;
  }
  if (level >= 0 && level < L && !c->solved) {
    c->err = "hhg_macro_norms with level < L needs a preceding successful hhg_fmg_solve";
    return HHG_ESTATE;
  }
  if ((level == L || !x) && !c->have_u) {
    c->err = "hhg_macro_norms needs u_L of a preceding successful solve";
    return HHG_ESTATE;
  }
  // only the scratch vectors rc and t are written: the last solve's u and w stay valid
  Level& lL = c->lev[L];
  const double* u = lL.x;
  if (x) {
    launch_canon_to_full(c->dim, lk_of(c, L), c->tab, x, lL.rc, 0, ST(c));
    u = lL.rc;
  }
  const double* a;
  if (level == -1) {
    launch_fill<double>(lL.t, lL.nfull, 0.0, ST(c));
    a = lL.t;
  } else if (level == L) {
    a = lL.x;
  } else if (level == L - 1) {
    a = lL.w;
  } else {
    a = prolong_chain(c, c->lev[level + 1].w, level + 1, L, false);
  }
  LAUNCHCHK();
  std::vector<double> s1, s2;
  // the kernel's second norm (against a level L-1 vector) is not used here
  TRY(estimate_pair(c, norm, a, c->lev[L - 1].x, s1, s2, u));
  for (int64_t m = 0; m < c->nC; ++m) sq[m] = s1[m];
  return HHG_OK;
}

hhg_status hhg_estimate(hhg_ctx c, int j, double* eta_cell, double* eta_j, double* theta_est, double* norm_e) {
  return hhg_estimate_ex(c, j, HHG_NORM_L2, HHG_LOCAL_L1, eta_cell, eta_j, theta_est, norm_e);
}

hhg_status hhg_apply(hhg_ctx c, int level, int op, const double* x, double* y) {
  TRY(check_ready(c));
  if (level < 0 || level > c->L || (op != HHG_OP_STIFFNESS && op != HHG_OP_MASS) || !x || !y) {
    c->err = "invalid argument";
    return HHG_EINVAL;
  }
  Level& lv = c->lev[level];
  launch_canon_to_full(c->dim, lk_of(c, level), c->tab, x, lv.rc, 0, ST(c));
  launch_apply<double, double>(c->dim, op == HHG_OP_STIFFNESS && p1(c), lk_of(c, level), c->tab, lv.rc, nullptr, lv.t,
                               op == HHG_OP_STIFFNESS ? 0 : 1, op == HHG_OP_STIFFNESS ? sA(c, level) : sM(c, level), 0.0,
                               1.0, 0, lv.kn, ST(c));
  launch_full_to_canon(c->dim, lk_of(c, level), c->tab, lv.t, y, 1, ST(c));
  LAUNCHCHK();
  // only the scratch vectors rc and t of the level are touched: the last solve's u and w stay
  // valid for hhg_estimate
  return HHG_OK;
}

hhg_status hhg_mass_apply(hhg_ctx c, const double* x, double* y) {
  if (!c) return HHG_EINVAL;
  return hhg_apply(c, c->L, HHG_OP_MASS, x, y);
}

hhg_status hhg_smooth(hhg_ctx c, int level, double* u, const double* b, int sweeps) {
  TRY(check_ready(c));
  if (level < 1 || level > c->L || !u || !b || sweeps < 0) { c->err = "invalid argument"; return HHG_EINVAL; }
  Level& lv = c->lev[level];
  launch_canon_to_full(c->dim, lk_of(c, level), c->tab, u, lv.x, 0, ST(c));
  launch_canon_to_full(c->dim, lk_of(c, level), c->tab, b, lv.rc, 1, ST(c));
  LAUNCHCHK();
  TRY(smooth<double>(c, level, lv.rc, sweeps));
  launch_full_to_canon(c->dim, lk_of(c, level), c->tab, lv.x, u, 0, ST(c));
  LAUNCHCHK();
  c->solved = false;
  c->have_u = false;
  return HHG_OK;
}

hhg_status hhg_restrict(hhg_ctx c, int level, const double* rf, double* rcn) {
  TRY(check_ready(c));
  if (level < 1 || level > c->L || !rf || !rcn) { c->err = "invalid argument"; return HHG_EINVAL; }
  Level& lf = c->lev[level];
  Level& lc = c->lev[level - 1];
  launch_canon_to_full(c->dim, lk_of(c, level), c->tab, rf, lf.t, 2, ST(c));
  launch_restrict<double>(c->dim, lk_of(c, level), lk_of(c, level - 1), c->tab, lf.t, lc.rc, ST(c));
  launch_full_to_canon(c->dim, lk_of(c, level - 1), c->tab, lc.rc, rcn, 1, ST(c));
  LAUNCHCHK();
  c->solved = false;
  c->have_u = false;
  return HHG_OK;
}

hhg_status hhg_prolongate(hhg_ctx c, int level, const double* ec, double* ef) {
  TRY(check_ready(c));
  if (level < 1 || level > c->L || !ec || !ef) { c->err = "invalid argument"; return HHG_EINVAL; }
  Level& lf = c->lev[level];
  Level& lc = c->lev[level - 1];
  launch_canon_to_full(c->dim, lk_of(c, level - 1), c->tab, ec, lc.rc, 0, ST(c));
  launch_prolong<double>(c->dim, lk_of(c, level), lk_of(c, level - 1), c->tab, lc.rc, lf.t, (double*)nullptr,
                         (const double*)nullptr, 1, ST(c));
  launch_full_to_canon(c->dim, lk_of(c, level), c->tab, lf.t, ef, 0, ST(c));
  LAUNCHCHK();
  c->solved = false;
  c->have_u = false;
  return HHG_OK;
}

hhg_status hhg_adjoint(hhg_ctx c, const double* f, const double* g, const double* dJdu, double* dJdf, double* dJdk,
                       const hhg_solve_params* p) {
  TRY(check_ready(c));
  TRY(validate_params(c, p));
  if (!f || !g || !dJdu) { c->err = "NULL vector"; return HHG_EINVAL; }
  const int L = c->L;
  Level& lL = c->lev[L];
  // 1. recompute u (nothing from the forward pass is stored)
  TRY(ensure_dense(c, *p));
  TRY(setup_rhs(c, f, g));
  TRY(fmg_core(c, *p, nullptr));
  launch_copy(c->d_aux0, lL.x, lL.nfull, ST(c));   // keep u
  // 2. adjoint right-hand side on level L (dual, Dirichlet rows zero), restricted downwards
  launch_canon_to_full(c->dim, lk_of(c, L), c->tab, dJdu, lL.bf, 2, ST(c));
  for (int l = L; l >= 1; --l)
    launch_restrict<double>(c->dim, lk_of(c, l), lk_of(c, l - 1), c->tab, c->lev[l].bf, c->lev[l - 1].bf, ST(c));
  for (int l = 0; l <= L; ++l) launch_fill<double>(c->lev[l].g, c->lev[l].nfull, 0.0, ST(c));
  LAUNCHCHK();
  // 3. lambda by FMG + extra cycles (homogeneous Dirichlet data)
  TRY(fmg_core(c, *p, nullptr));
  // 4. dJ/df = M lambda
  if (dJdf) {
    launch_apply<double, double>(c->dim, false, lk_of(c, L), c->tab, lL.x, nullptr, lL.t, 1, sM(c, L), 0.0, 1.0, 0,
                                 nullptr, ST(c));
    launch_full_to_canon(c->dim, lk_of(c, L), c->tab, lL.t, dJdf, 1, ST(c));
  }
  // 5. dJ/dkappa_e = -lambda^T A_e u
  if (dJdk) {
    double* out = c->d_red + (c->red_capacity - c->nC - 8);
    launch_bilinear(c->dim, lk_of(c, L), c->tab, lL.x, c->d_aux0, c->d_red, out, sA(c, L), ST(c));
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(dJdk, out, c->nC * 8, hipMemcpyDeviceToHost, ST(c)));
    HIPCHK(hipStreamSynchronize(ST(c)));
    for (int64_t m = 0; m < c->nC; ++m) dJdk[m] = -dJdk[m];
  }
  LAUNCHCHK();
  c->solved = false;
  c->have_u = false;
  return HHG_OK;
}

hhg_status hhg_bench_smoother(hhg_ctx c, int precision, int sweeps, double* ms, double* bytes, double* launch_ms,
                              double* launch_bytes) {
  TRY(check_ready(c));
  if (sweeps < 1 || (precision != HHG_FP64 && precision != HHG_FP32_REFINED)) { c->err = "invalid argument"; return HHG_EINVAL; }
  const int L = c->L;
  Level& lL = c->lev[L];
  // events around every finest-level interior launch of the timed sweeps
  const int need = 2 * sweeps * std::max(lL.ncolours, 1);
  while ((int)c->prof_ev.size() < need) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    c->prof_ev.push_back(e);
  }
  TRY(ensure_events(c));
  c->prof_used = 0;
  c->prof_bytes = 0.0;
  c->prof_on = launch_ms != nullptr || launch_bytes != nullptr;
  HIPCHK(hipEventRecord((hipEvent_t)c->ev0, ST(c)));
  hhg_status s = precision == HHG_FP64 ? smooth<double>(c, L, lL.bf, sweeps) : smooth<float>(c, L, lL.b32, sweeps);
  c->prof_on = false;
  TRY(s);
  HIPCHK(hipEventRecord((hipEvent_t)c->ev1, ST(c)));
  HIPCHK(hipEventSynchronize((hipEvent_t)c->ev1));
  float t = 0;
  HIPCHK(hipEventElapsedTime(&t, (hipEvent_t)c->ev0, (hipEvent_t)c->ev1));
  if (ms) *ms = t;
  const double per = precision == HHG_FP64 ? 24.0 + (p1(c) ? 8.0 : 0.0) : 12.0 + (p1(c) ? 8.0 : 0.0);
  if (bytes) *bytes = per * (double)lL.ndof * sweeps;
  const int pairs = c->prof_used / 2;
  double tot = 0.0;
  for (int q = 0; q < pairs; ++q) {
    float e = 0;
    HIPCHK(hipEventElapsedTime(&e, (hipEvent_t)c->prof_ev[2 * q], (hipEvent_t)c->prof_ev[2 * q + 1]));
    tot += e;
  }
  if (launch_ms) *launch_ms = pairs ? tot / pairs : 0.0;
  if (launch_bytes) *launch_bytes = pairs ? c->prof_bytes / pairs : 0.0;
  c->solved = false;
  c->have_u = false;
  return HHG_OK;
}

hhg_status hhg_residual_history(hhg_ctx c, double* out, int capacity, int* count) {
  if (!c || !count || capacity < 0 || (capacity > 0 && !out)) return HHG_EINVAL;
  const int n = (int)c->res_hist.size();
  *count = n;
  for (int q = 0; q < std::min(n, capacity); ++q) out[q] = c->res_hist[q];
  return HHG_OK;
}

void hhg_destroy(hhg_ctx c) {
  if (!c) return;
  // recorded launches may still run: finish them before their executable graphs go
  if (c->bound) (void)hipStreamSynchronize(ST(c));
  release_static(c);
  drop_graphs(c);
  if (c->cap_stream) (void)hipStreamDestroy((hipStream_t)c->cap_stream);
  for (void* e : c->prof_ev) (void)hipEventDestroy((hipEvent_t)e);
  if (c->ev0) (void)hipEventDestroy((hipEvent_t)c->ev0);
  if (c->ev1) (void)hipEventDestroy((hipEvent_t)c->ev1);
  delete c;
}

}  // extern "C"
