// Launch interface of the HHG kernels (hhg_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hhg_internal.h"

namespace hhg {

// level descriptor passed to kernels by value
struct LK {
  int n = 1, l = 0;
  int64_t S = 0;
  int Sraw = 0, NI = 0, nEd = 0, nFd = 0;
  int64_t nIface = 0, ndof = 0;
  int nmacro = 0;
  int rows3d_min = 128;   // 3D levels with n >= this use the row kernels
  int planes3d = 0;       // 3D: the level's tiles are chunks of the whole-plane sweep
};

template <typename T>
void launch_smooth_interior(int dim, bool p1, const LK& lk, const Tables& tb, const T* uin, T* uout, const T* b, int colour,
                            int rb, int jacobi, double omega, double sA, const double* kn, bool fine, hipStream_t st);
// fused interior Gauss-Seidel sweep (all interior colours); false if not available for the level
// (2D, and 3D with streaming tiles: reads u and writes the interior of uo; the 3D LDS macro
// sweep updates u in place and ignores uo).  2D with pro_ec: the sweep starts from u + P pro_ec
// (the prolongation of the coarse correction pro_ec, coarse closure stride pro_cS) and writes
// that start value of every macro-boundary node to pro_t; with zero_start instead, it starts
// from zero (u is not read) and writes zeros to the macro-boundary nodes of pro_t
template <typename T>
bool launch_gs_fused(int dim, bool p1, const LK& lk, const Tables& tb, T* u, T* uo, const T* b, const int32_t* tiles,
                     int ntiles, const uint32_t* itab, const int32_t* itab_off, int rb, double sA, bool fine,
                     hipStream_t st, const T* pro_ec = nullptr, int pro_cS = 0, T* pro_t = nullptr,
                     bool zero_start = false);
// interface update of one colour class (xi: source of interior neighbours, xf: of interface
// neighbours; umirror, if not NULL, receives the new values too)
// lane-parallel interface update of the wavefronts w0..w1-1 (one colour class), or of all
// classes c0..c1-1 in one workgroup
template <typename T>
void launch_iface_tasks(int dim, const LK& lk, const Tables& tb, const int32_t* tp, const int32_t* tq, const int32_t* tco,
                        const int32_t* tseg, const int32_t* wmax, int w0, int w1, const T* xi, const T* xf, T* uout,
                        T* umirror, const T* b, int jacobi, double omega, double sA, hipStream_t st);
template <typename T>
void launch_iface_tasks_1wg(int dim, const LK& lk, const Tables& tb, const int32_t* tp, const int32_t* tq,
                            const int32_t* tco, const int32_t* tseg, const int32_t* wmax, const int32_t* woff, int c0,
                            int c1, const T* xi, const T* xf, T* uout, T* umirror, const T* b, double sA, bool pre,
                            hipStream_t st, int sweeps = 1);
// 2D: both edge classes of a sweep in one launch (edge chunks; erec: one record of
// kEdgeRecWords words per macro edge), plus the copies of the Dirichlet vertex values
template <typename T>
void launch_iface2d_edges(const LK& lk, const int32_t* erec, int nE, const int32_t* dvcopy, int n_dv, const T* xi,
                          const T* xf, T* uout, T* umirror, const T* b, double sA, hipStream_t st);
// 2D: the vertex classes c_vr0 .. c_vr0 + ncls - 1 of a sweep by wheels, one launch
template <typename T>
void launch_iface2d_wheels(const LK& lk, const Tables& tb, const int32_t* wcopy, const int32_t* winfo,
                           const int32_t* wloc, const int32_t* wseg, const int32_t* wsrc, const double* wcw,
                           const int32_t* wwmax, int nwaves, int ncls, const T* xi, const T* xf, T* uout, T* umirror,
                           const T* b, double sA, hipStream_t st);
// 2D, out of place: both edge classes and all vertex classes of a sweep in one launch (the
// wheels recompute their edge-class neighbours; we2: per wheel lane the edge, side and
// direction of that neighbour, or -1; a2i, a2w: that neighbour's rows, 16 entries per lane as a
// struct of arrays); no mirror writes
template <typename T>
void launch_iface2d_sweep(const LK& lk, const Tables& tb, const int32_t* erec, int nE, const int32_t* dvcopy, int n_dv,
                          const int32_t* wcopy, const int32_t* winfo, const int32_t* wloc, const int32_t* wseg,
                          const int32_t* wsrc, const double* wcw, const int32_t* wwmax, int nwaves, int ncls,
                          const int32_t* we2, const int32_t* a2i, const double* a2w, const T* xi, const T* xf,
                          T* uout, const T* b, double sA, hipStream_t st);
// classes the preloading single-workgroup interface form holds at once
int iface_pre_classes(int dim, bool dbl);
template <typename T>
void launch_smooth_iface(int dim, bool p1, const LK& lk, const Tables& tb, const int32_t* list, int count, const T* xi,
                         const T* xf, T* uout, T* umirror, const T* b, int jacobi, double omega, double sA,
                         const double* kn, hipStream_t st);
// interface classes c0..c1-1 in one single-workgroup launch
template <typename T>
void launch_iface_sweep_1wg(int dim, bool p1, const LK& lk, const Tables& tb, const int32_t* list, const int32_t* coff,
                            int c0, int c1, const T* xi, const T* xf, T* uout, T* umirror, const T* b, double sA,
                            const double* kn, hipStream_t st);
template <typename Tin, typename Tout>
void launch_apply(int dim, bool p1, const LK& lk, const Tables& tb, const Tin* x, const Tin* b, Tout* y, int op,
                  double scale, double alpha, double beta, int zero_dir, const double* kn, hipStream_t st);
// interface residual rows from the interface tasks (wavefronts w0..w1-1 of all classes)
template <typename Tin, typename Tout>
void launch_iface_residual_tasks(int dim, const LK& lk, const Tables& tb, const int32_t* tp, const int32_t* tq,
                                 const int32_t* tco, const int32_t* tseg, const int32_t* wmax, int w0, int w1,
                                 const Tin* x, const Tin* b, Tout* y, double sA, hipStream_t st);
template <typename Tin, typename Tout>
void launch_iface_residual(int dim, bool p1, const LK& lk, const Tables& tb, const Tin* x, const Tin* b, Tout* y,
                           double sA, const double* kn, hipStream_t st);
template <typename T>
void launch_restrict(int dim, const LK& f, const LK& c, const Tables& tb, const T* rf, T* bc, hipStream_t st,
                     T* zc = nullptr);
template <typename T>
void launch_prolong(int dim, const LK& f, const LK& c, const Tables& tb, const T* ec, T* uf, T* w, const T* g, int mode,
                    hipStream_t st);
void launch_inject(int dim, const LK& fine, const LK& coarse, const double* src, double* dst, hipStream_t st);
void launch_init_dirichlet(int dim, const LK& lk, const Tables& tb, const double* g, double* x, double inner,
                           hipStream_t st);
template <typename T>
void launch_coarse(int n0, const int32_t* coff, const int64_t* copy, const double* Ainv, const T* rhs, T* x, int accumulate,
                   hipStream_t st);
// level 0 in factored form: x (+)= P^T X^T X P rhs (scr: 2 n0 doubles of scratch)
template <typename T>
void launch_coarse_factored(int n0, const int32_t* coff, const int64_t* copy, const int32_t* perm, const double* X,
                            double* scr, const T* rhs, T* x, int accumulate, hipStream_t st);
// dense map of the coarse cycle: sum[c] = sum of b (nb entries) over the copies of DoF c (gather
// table gat, kmax copies at most), then x[copies of DoF r] = sum_c B[r][c] sum[c] (ld a multiple
// of 256, at most 8192); its probes: b = unit vector at idx, and the probe's result x written
// into column `probe` of B
template <typename T>
void launch_dense_map(int rows, int ld, int kmax, const int32_t* gat, T* sum, const T* B, const T* b, int64_t nb,
                      const int32_t* off, const int32_t* copy, T* x, hipStream_t st);
template <typename T>
void launch_unit(T* b, int64_t n, int64_t idx, hipStream_t st);
template <typename T>
void launch_dense_harvest(int rows, const int32_t* off, const int32_t* copy, int ld, int probe, const T* x, T* B,
                          hipStream_t st);
void launch_sqnorm(int dim, const LK& lk, const Tables& tb, const double* r, double* partial, double* out, hipStream_t st);
// sum of squares of every closure entry (interface rows assembled in one copy)
template <typename T>
void launch_sqnorm_closure(int dim, const LK& lk, const T* r, double* partial, double* out, hipStream_t st);
// per-macro squared norms of u - a and u - P bc; norm 0 = consistent mass (scale sM),
// 1 = stiffness with the macro coefficients (scale sA), 2 = lumped mass (scale sM)
void launch_estimate(int dim, int norm, const LK& f, const LK& c, const Tables& tb, const double* u, const double* a,
                     const double* bc, double* partial, double* out, double scale, bool rows, hipStream_t st);
void launch_bilinear(int dim, const LK& lk, const Tables& tb, const double* x, const double* y, double* partial,
                     double* out, double sA, hipStream_t st);
void launch_canon_to_full(int dim, const LK& lk, const Tables& tb, const double* canon, double* full, int mode,
                          hipStream_t st);
void launch_full_to_canon(int dim, const LK& lk, const Tables& tb, const double* full, double* canon, int mode,
                          hipStream_t st);
void launch_dof_coords(int dim, const LK& lk, const Tables& tb, const double* mxyz, const int32_t* cells, double* xyz,
                       hipStream_t st);
template <typename T>
void launch_fill(T* x, int64_t n, T v, hipStream_t st);
void launch_add_f32(double* u, const float* e, int64_t n, hipStream_t st);
void launch_copy(double* dst, const double* src, int64_t n, hipStream_t st);

// x = g on Dirichlet nodes of a level, other nodes unchanged
void launch_impose_dirichlet(int dim, const LK& lk, const Tables& tb, const double* g, double* x, hipStream_t st);
// 2D transfer of a level vector (closure layout) from old macros to the closure nodes of new
// macros; candidate old macros of new macro m: cand[coff[m] .. coff[m+1]-1]
void launch_transfer(int dim, const LK& fn, const double* mxyz_new, const LK& fo, const double* mxyz_old,
                     const int32_t* coff, const int32_t* cand, const double* uold, double* unew, hipStream_t st);

}  // namespace hhg
