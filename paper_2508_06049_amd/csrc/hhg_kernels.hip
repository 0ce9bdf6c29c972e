// HIP kernels of the HHG library for gfx950 (wave64).
//
// Data layout (see hhg_internal.h): every level vector is stored per macro element over its
// whole closure, so a micro node on a macro vertex, edge or face has one copy per adjacent
// macro.  Two kinds of vectors live in this layout:
//   primal (solutions, corrections, nodal data): all copies hold the same value;
//   dual (right-hand sides, residuals): copies hold per-macro partial sums whose total is the
//        assembled value (each macro contributes the rows of its own micro elements).
// With this split the residual, the restriction P^T, the prolongation P and the mass/stiffness
// products are purely macro-local; only the smoother's interface update and the norms sum
// over the copies of a DoF (additive collection from the adjacent volume macros, Section 4.4).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hhg_internal.h"
#include "hhg_kernels.h"
#include "hhg_lattice.h"

namespace hhg {

// ------------------------------------------------------------------------------------------
// index helpers
__device__ __forceinline__ int d_tet(int m) { return m < 0 ? 0 : ((m + 1) * (m + 2) * (m + 3)) / 6; }
__device__ __forceinline__ int d_lin2(int n, int i, int j) { return j * (n + 1) - (j * (j - 1)) / 2 + i; }

template <int D>
__device__ __forceinline__ int d_lin(int n, int i, int j, int k) {
  if constexpr (D == 2) {
    return d_lin2(n, i, j);
  } else {
    const int m = n - k;
    return d_tet(n) - d_tet(m) + d_lin2(m, i, j);
  }
}

// row j of linear index s in a triangle of side n: a single-precision estimate from the
// quadratic row-offset formula, then exact integer correction
__device__ __forceinline__ void d_dec2(int n, int s, int& i, int& j) {
  const float a = 2.0f * (float)n + 3.0f;
  int jj = (int)floorf(0.5f * (a - sqrtf(fmaxf(a * a - 8.0f * (float)s, 0.0f))));
  jj = max(0, min(jj, n));
  while (jj < n && d_lin2(n, 0, jj + 1) <= s) ++jj;
  while (jj > 0 && d_lin2(n, 0, jj) > s) --jj;
  j = jj;
  i = s - d_lin2(n, 0, jj);
}

template <int D>
__device__ __forceinline__ void d_dec(int n, int s, int& i, int& j, int& k) {
  if constexpr (D == 2) {
    k = 0;
    d_dec2(n, s, i, j);
  } else {
    const int r = d_tet(n) - s;   // >= 1
    int m = (int)cbrtf(6.0f * (float)r) - 2;
    m = max(0, min(m, n));
    while (d_tet(m) < r) ++m;
    while (m > 0 && d_tet(m - 1) >= r) --m;
    k = n - m;
    d_dec2(m, s - (d_tet(n) - d_tet(m)), i, j);
  }
}

template <int D>
__device__ __forceinline__ int d_mask(int n, int i, int j, int k) {
  const int c0 = n - i - j - (D == 3 ? k : 0);
  int mk = (c0 == 0 ? 1 : 0) | (i == 0 ? 2 : 0) | (j == 0 ? 4 : 0);
  if constexpr (D == 3) mk |= (k == 0 ? 8 : 0);
  return mk;
}

template <int D>
__device__ __forceinline__ void d_off(int q, int& a, int& b, int& c) {
  if constexpr (D == 3) {
    a = kOff3[q][0]; b = kOff3[q][1]; c = kOff3[q][2];
  } else {
    a = kOff2[q][0]; b = kOff2[q][1]; c = 0;
  }
}

template <int D>
__device__ __forceinline__ void d_typeoff(int t, int v, int& a, int& b, int& c) {
  if constexpr (D == 3) {
    a = kType3[t][v][0]; b = kType3[t][v][1]; c = kType3[t][v][2];
  } else {
    a = kType2[t][v][0]; b = kType2[t][v][1]; c = 0;
  }
}

// raw buffer access to one block (a macro's, or a whole level vector): a descriptor plus a
// 32-bit per-lane byte offset, so address arithmetic costs one VGPR per access.  The
// descriptor's size bounds the access: loads past it return 0 and stores are dropped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t d_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ void d_bload(__amdgpu_buffer_rsrc_t r, uint32_t off, float& v) {
  v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ void d_bload(__amdgpu_buffer_rsrc_t r, uint32_t off, double& v) {
  v = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void d_bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 0);
}
__device__ __forceinline__ void d_bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v),
                                        r, off, 0, 0);
}

template <int D> constexpr int ndir() { return D == 3 ? kNDir3 : kNDir2; }
template <int D> constexpr int ntype() { return D == 3 ? kNType3 : kNType2; }

// block-wide sum of one double (blockDim.x == 256, wave64)
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return r;
}

// Logical block of this workgroup for kernels whose consecutive logical blocks touch the same
// data (one macro's chunks, one class's wavefronts): block b runs on XCD b mod 8, so XCD x takes
// the logical blocks x * per .. (x + 1) * per - 1 and their shared lines stay in one L2.  The
// grid is padded to a multiple of 8 (grid8); logical blocks past the end return.
__device__ __forceinline__ int d_xcd_block() {
  const int per = (int)(gridDim.x >> 3);
  return (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
}

// interface DoF t -> primitive p and coordinates along its sorted vertices
__device__ __forceinline__ void d_iface_decode(const LK& lk, const Tables& tb, int64_t t, int& p, int co[3], int& np) {
  const int n = lk.n;
  co[0] = co[1] = co[2] = 0;
  if (t < tb.nV) { p = (int)t; co[0] = n; np = 1; return; }
  t -= tb.nV;
  if (t < (int64_t)tb.nE * lk.nEd) {
    p = tb.nV + (int)(t / lk.nEd);
    const int a = (int)(t % lk.nEd) + 1;
    co[0] = n - a; co[1] = a; np = 2;
    return;
  }
  t -= (int64_t)tb.nE * lk.nEd;
  p = tb.nV + tb.nE + (int)(t / lk.nFd);
  int a, b;
  d_dec2(n - 3, (int)(t % lk.nFd), a, b);
  co[1] = a + 1; co[2] = b + 1; co[0] = n - co[1] - co[2]; np = 3;
}

// canonical DoF index of closure point (i,j,k) of macro m
template <int D>
__device__ __forceinline__ int64_t d_canon(const LK& lk, const Tables& tb, int m, int i, int j, int k) {
  const int n = lk.n;
  const int mask = d_mask<D>(n, i, j, k);
  if (mask == 0) return lk.nIface + (int64_t)m * lk.NI + d_lin<D>(n - D - 1, i - 1, j - 1, k - 1);
  const int p = tb.subprim[m * kMaxMask + mask];
  const int ord = tb.suborder[m * kMaxMask + mask];
  const int cc[4] = {n - i - j - (D == 3 ? k : 0), i, j, k};
  if (p < tb.nV) return p;
  if (p < tb.nV + tb.nE) return tb.nV + (int64_t)(p - tb.nV) * lk.nEd + (cc[(ord >> 2) & 3] - 1);
  const int a = cc[(ord >> 2) & 3], b = cc[(ord >> 4) & 3];
  return tb.nV + (int64_t)tb.nE * lk.nEd + (int64_t)(p - tb.nV - tb.nE) * lk.nFd + d_lin2(n - 3, a - 1, b - 1);
}

// value of P e_c at fine closure point (i,j,k) (fine n), coarse vector with macro base cbase
template <int D, typename T>
__device__ __forceinline__ T d_prolong_val(int nc, const T* __restrict__ ec, int64_t cbase, int i, int j, int k) {
  const int p = (i & 1) | ((j & 1) << 1) | ((D == 3 ? (k & 1) : 0) << 2);
  if (p == 0) return ec[cbase + d_lin<D>(nc, i >> 1, j >> 1, k >> 1)];
  int a, b, c;
  if constexpr (D == 3) { a = kParDir3[p][0]; b = kParDir3[p][1]; c = kParDir3[p][2]; }
  else { a = kParDir2[p][0]; b = kParDir2[p][1]; c = 0; }
  const T lo = ec[cbase + d_lin<D>(nc, (i - a) >> 1, (j - b) >> 1, (k - c) >> 1)];
  const T hi = ec[cbase + d_lin<D>(nc, (i + a) >> 1, (j + b) >> 1, (k + c) >> 1)];
  return (T)0.5 * (lo + hi);
}

// closure index of the neighbour of (i,j,k) in 3D direction q (kOff3), from the plane and row
// offsets of the point: the 14 neighbours lie on 7 rows (row j + b of plane k + c), and with
// P(k) the first point of plane k and r = rowin(j, k) = j (n - k + 1) - j (j - 1) / 2,
// rowin(j + 1, k) = r + (n - k + 1) - j, rowin(j, k + 1) = r - j, P(k + 1) = P(k) + (n - k + 1)
// (n - k + 2) / 2.  Only neighbours inside the closure are meaningful.
struct Nbr3 {
  int c00, cp0, cm0, c0p, c0m, cmp, cpm;   // row starts + i of the rows (b, c) = (0,0) (1,0) (-1,0) (0,1) (0,-1) (-1,1) (1,-1)
  __device__ __forceinline__ Nbr3(int n, int i, int j, int k) {
    const int pk = d_tet(n) - d_tet(n - k);
    const int n1 = n - k + 1;
    const int r = j * n1 - ((j * (j - 1)) >> 1);
    const int pp = pk + ((n1 * (n1 + 1)) >> 1), pm = pk - (((n1 + 1) * (n1 + 2)) >> 1);
    c00 = pk + r + i;
    cp0 = c00 + n1 - j;
    cm0 = c00 - n1 + j - 1;
    c0p = pp + r - j + i;
    c0m = pm + r + j + i;
    cmp = pp + r - n1 + i;
    cpm = pm + r + n1 + 1 + i;
  }
  __device__ __forceinline__ int at(int q) const {
    const int b = kOff3[q][1], c = kOff3[q][2], a = kOff3[q][0];
    const int rb = c == 0 ? (b == 0 ? c00 : (b > 0 ? cp0 : cm0)) : (c > 0 ? (b == 0 ? c0p : cmp) : (b == 0 ? c0m : cpm));
    return rb + a;
  }
};

// closure index of the neighbour in direction q of a 2D or 3D closure point
template <int D>
struct NbrIdx;
template <>
struct NbrIdx<3> : Nbr3 {
  __device__ __forceinline__ NbrIdx(int n, int i, int j, int k) : Nbr3(n, i, j, k) {}
};
template <>
struct NbrIdx<2> {
  int n, i, j;
  __device__ __forceinline__ NbrIdx(int n_, int i_, int j_, int) : n(n_), i(i_), j(j_) {}
  __device__ __forceinline__ int at(int q) const { return d_lin2(n, i + kOff2[q][0], j + kOff2[q][1]); }
};

// row of the partial operator of macro m at closure point (i,j,k) with zero-set `mask`:
// off = sum_{neighbours} a_q x_q, diag = a_centre.  Constant-coefficient stencil table.
template <int D, typename T>
__device__ __forceinline__ void d_row_const(const LK& lk, const double* __restrict__ W, uint32_t valid, double scale,
                                            const T* __restrict__ x, int64_t base, int i, int j, int k, T& off, T& diag) {
  constexpr int ND = ndir<D>();
  T acc = (T)0;
  if constexpr (D == 3) {
    const Nbr3 nb(lk.n, i, j, k);
#pragma unroll
    for (int q = 1; q < ND; ++q) {
      if (!((valid >> q) & 1)) continue;
      acc += (T)(scale * W[q]) * x[base + nb.at(q)];
    }
  } else {
#pragma unroll
    for (int q = 1; q < ND; ++q) {
      if (!((valid >> q) & 1)) continue;
      int a, b, c;
      d_off<D>(q, a, b, c);
      acc += (T)(scale * W[q]) * x[base + d_lin<D>(lk.n, i + a, j + b, k + c)];
    }
  }
  off = acc;
  diag = (T)(scale * W[0]);
}

// same with a nodal coefficient: every incident micro element contributes with the mean of
// the nodal coefficient over its vertices
template <int D, typename T>
__device__ __forceinline__ void d_row_p1(const LK& lk, const double* __restrict__ EK, uint32_t incvalid, double scale,
                                         const double* __restrict__ kn, const T* __restrict__ x, int64_t base, int i,
                                         int j, int k, T& off, T& diag) {
  constexpr int NV = D + 1, NT = ntype<D>();
  T acc = (T)0, dg = (T)0;
  for (int t = 0; t < NT; ++t) {
#pragma unroll
    for (int a = 0; a < NV; ++a) {
      if (!((incvalid >> (t * NV + a)) & 1)) continue;
      int oa0, oa1, oa2;
      d_typeoff<D>(t, a, oa0, oa1, oa2);
      int idx[NV];
      double ks = 0.0;
#pragma unroll
      for (int b = 0; b < NV; ++b) {
        int o0, o1, o2;
        d_typeoff<D>(t, b, o0, o1, o2);
        idx[b] = d_lin<D>(lk.n, i + o0 - oa0, j + o1 - oa1, k + o2 - oa2);
        ks += kn[base + idx[b]];
      }
      ks *= scale / NV;
      const double* Kr = EK + (t * NV + a) * NV;
#pragma unroll
      for (int b = 0; b < NV; ++b) {
        if (b == a) dg += (T)(ks * Kr[b]);
        else acc += (T)(ks * Kr[b]) * x[base + idx[b]];
      }
    }
  }
  off = acc;
  diag = dg;
}

// ------------------------------------------------------------------------------------------
// smoothers
// FINE only labels the launches on the finest level (separate profiler statistics)
template <int D, typename T, bool P1, bool FINE>
__global__ void __launch_bounds__(256) k_smooth_interior(LK lk, Tables tb, const T* __restrict__ uin, T* __restrict__ uout,
                                                          const T* __restrict__ b, int colour, int rb, int jacobi,
                                                          double omega, double sA, const double* __restrict__ kn) {
  const int nchunk = (lk.NI + 255) >> 8;
  const int blk = d_xcd_block();
  const int m = blk / nchunk;
  const int s = (blk - m * nchunk) * 256 + threadIdx.x;
  if (m >= lk.nmacro || s >= lk.NI) return;
  int i, j, k;
  d_dec<D>(lk.n - D - 1, s, i, j, k);
  ++i; ++j;
  if constexpr (D == 3) ++k;
  if (!jacobi) {
    int c;
    if (rb) {
      const int* rp = tb.rbpar + m * 4;
      c = (i * rp[1] + j * rp[2] + (D == 3 ? k * rp[3] : 0)) & 1;
    } else {
      c = D == 2 ? (i + 2 * j) % 3 : (i + 2 * j + 3 * k) % 4;
    }
    if (c != colour) return;
  }
  const int64_t base = (int64_t)m * lk.S;
  const int ctr = d_lin<D>(lk.n, i, j, k);
  T off, diag;
  if constexpr (P1) {
    d_row_p1<D, T>(lk, tb.elemK + (size_t)m * ntype<D>() * (D + 1) * (D + 1), tb.incvalid[0], sA, kn, uin, base, i, j, k,
                   off, diag);
  } else {
    d_row_const<D, T>(lk, tb.stiff + (size_t)m * kMaxMask * ndir<D>(), tb.validdirs[0], sA * tb.kappa[m], uin, base, i,
                      j, k, off, diag);
  }
  if (jacobi) {
    const T u0 = uin[base + ctr];
    uout[base + ctr] = u0 + (T)omega * (b[base + ctr] - off - diag * u0) / diag;
  } else {
    uout[base + ctr] = (b[base + ctr] - off) / diag;
  }
}

// 3D interior Gauss-Seidel of one colour class by rows: one wavefront per interior row (j, k)
// of one macro (j, k >= 1, j + k <= n - 2), lanes along i in segments of 64.  The macro, the
// row and the offsets of the 14 neighbour rows are wave-uniform and computed once; stencil
// weights that vanish (the 7-point stencils of Kuhn macros) are skipped for the whole wave.
// Rows are numbered plane by plane (k, then j), so the neighbour rows of a wavefront are
// swept by wavefronts close to it in time; blocks are spread over the XCDs in contiguous runs
// (block b runs on XCD b mod 8).  Same update, in the same order, as k_smooth_interior.
template <typename T, bool FINE>
__global__ void __launch_bounds__(256) k_gs3d_rows(LK lk, Tables tb, T* __restrict__ u, const T* __restrict__ b,
                                                    int colour, int rb, double sA, int nrows) {
  const int per_xcd = (int)(gridDim.x >> 3);   // gridDim.x is a multiple of 8
  const int blk = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  const int wid = __builtin_amdgcn_readfirstlane(blk * 4 + (int)(threadIdx.x >> 6));
  if (wid >= lk.nmacro * nrows) return;
  const int n = lk.n;
  const int m = wid / nrows;
  const int r = wid - m * nrows;
  // plane k holds the rows j = 1 .. n - 2 - k: r = sum_{k' < k} (n - 2 - k') + (j - 1)
  const float a = 2.0f * (float)n - 5.0f;
  int k = 1 + (int)floorf(0.5f * (a - sqrtf(fmaxf(a * a - 8.0f * (float)r, 0.0f))));
  k = max(1, min(k, n - 3));
  auto first = [&](int kk) { return (kk - 1) * (n - 2) - ((kk - 1) * kk) / 2; };
  while (k < n - 3 && first(k + 1) <= r) ++k;
  while (k > 1 && first(k) > r) --k;
  const int j = 1 + r - first(k);
  const int64_t base = (int64_t)m * lk.S;
  auto row = [&](int jj, int kk) { return d_tet(n) - d_tet(n - kk) + jj * (n - kk + 1) - (jj * (jj - 1)) / 2; };
  const double* W = tb.stiff + (size_t)m * kMaxMask * 15;
  const double ks = sA * tb.kappa[m];
  const T diag = (T)(ks * W[0]);
  const int len = n - 1 - j - k;   // interior points i = 1 .. len
  const int ctr0 = row(j, k);
  // the points of this colour along the row: i = i1, i1 + P, ... (period P in i)
  int i1, P;
  if (rb) {
    const int* rp = tb.rbpar + m * 4;
    const int c1 = (rp[1] + j * rp[2] + k * rp[3]) & 1;
    if (rp[1] & 1) {
      P = 2;
      i1 = c1 == colour ? 1 : 2;
    } else {
      if (c1 != colour) return;
      P = 1;
      i1 = 1;
    }
  } else {
    P = 4;
    i1 = 1 + ((colour - (1 + 2 * j + 3 * k)) % 4 + 4) % 4;
  }
  T cq[15];
  int64_t ro[15];
#pragma unroll
  for (int q = 1; q < 15; ++q) {
    cq[q] = (T)(ks * W[q]);
    ro[q] = base + row(j + kOff3[q][1], k + kOff3[q][2]) + kOff3[q][0];
  }
  const int lane = (int)(threadIdx.x & 63);
  for (int i = i1 + P * lane; i <= len; i += 64 * P) {
    T off = (T)0;
#pragma unroll
    for (int q = 1; q < 15; ++q) {
      if (W[q] == 0.0) continue;
      off += cq[q] * u[ro[q] + i];
    }
    const int64_t ctr = base + ctr0 + i;
    u[ctr] = (b[ctr] - off) / diag;
  }
}

// Red-black Gauss-Seidel sweep of all macro interiors of a 3D level, both colours in one
// launch, out of place: reads u, writes the interior of uo.  One workgroup takes a tile of
// kS3I x kS3J points in (i, j) and streams the planes k0 .. k1-1 of one macro.  Per plane p it
// loads u on the tile plus a two-point halo into LDS, updates the red points of plane p-1 on the
// tile plus a one-point halo (in place in LDS: red points read only black neighbours, and the
// black update reads only red ones), then the black points of plane p-2 on the tile, and writes
// both colours of plane p-2.  Red values at halo points are recomputed here, identically to the
// tile that owns them, since all their inputs are old values.  Per point this moves u and b once
// in and u once out (plus the halos, mostly served by L2).  Same updates, in the same order
// within each point, as the class-by-class sweep: red (parity 0) first, then black; interface
// points are left to the interface sweep.  The parity alternates along i on every macro of a
// level with streaming tiles, so every lane takes one (red, black) pair of neighbouring points
// and no lane idles in either colour phase.
template <typename T, bool FINE>
__global__ void __launch_bounds__(256) k_gs3d_stream(LK lk, Tables tb, const T* __restrict__ u, T* __restrict__ uo,
                                                     const T* __restrict__ b, const int32_t* __restrict__ tiles,
                                                     int ntiles, double sA) {
  constexpr int W = 64, H = kS3J + 4, NP = W * H / 256, NS = 5;
  constexpr int NQ = (H - 2) * (W / 2), RQ = (NQ + 255) / 256;   // point pairs of the halo rows
  static_assert(kS3I + 4 == W, "one wavefront per LDS row");
  __shared__ T sU[NS][H * W];   // u of five planes; red points updated in place
  const int per_xcd = (int)(gridDim.x >> 3);   // gridDim.x is a multiple of 8
  const int blk = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  if (blk >= lk.nmacro * ntiles) return;
  const int m = blk / ntiles;
  const int tile = tiles[blk - m * ntiles];
  const int n = lk.n;
  const int i0 = 1 + (tile & 1023) * kS3I, j0 = 1 + ((tile >> 10) & 1023) * kS3J, k0 = 1 + (tile >> 20) * kS3K;
  const int k1 = min(k0 + kS3K, n - i0 - j0);   // interior points with i >= i0, j >= j0 have k < n - i0 - j0
  // the macro's closure as buffer resources: 32-bit offsets, every access below stays inside
  const int64_t base = (int64_t)m * lk.S;
  const uint32_t mbytes = (uint32_t)(lk.S * (int64_t)sizeof(T));
  const __amdgpu_buffer_rsrc_t ru = d_rsrc(u + base, mbytes), rb = d_rsrc(b + base, mbytes),
                               ro = d_rsrc(uo + base, mbytes);
  const double* Wt = tb.stiff + (size_t)m * kMaxMask * 15;
  const double ks = sA * tb.kappa[m];
  const T diag = (T)(ks * Wt[0]);
  // all 14 neighbours are read and weighted, vanishing weights included: adding the exact zero
  // products leaves every sum bitwise as it is, and unconditional LDS reads stay in flight
  T cq[15];
#pragma unroll
  for (int q = 1; q < 15; ++q) cq[q] = (T)(ks * Wt[q]);
  const int* rp = tb.rbpar + m * 4;
  const int s1 = rp[1], s2 = rp[2], s3 = rp[3];
  const int tid = (int)threadIdx.x;
  const int lane = tid & 63, w4 = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int dn = d_tet(n);
  auto plane = [&](int k) { return dn - d_tet(n - k); };
  auto rowin = [&](int j, int k) { return j * (n - k + 1) - (j * (j - 1)) / 2; };
  auto slot = [](int k) { return (k + NS) % NS; };
  auto inner = [&](int i, int j, int k) { return i >= 1 && j >= 1 && k >= 1 && i + j + k <= n - 1; };
  auto col = [&](int i, int j, int k) { return (i * s1 + j * s2 + k * s3) & 1; };   // 0: red
  auto stencil = [&](const T* Um, const T* U0, const T* Up, int idx) {
    T nb[15];
#pragma unroll
    for (int c = 1; c < 15; ++c) {
      const T* P = kOff3[c][2] < 0 ? Um : (kOff3[c][2] > 0 ? Up : U0);
      nb[c] = P[idx + kOff3[c][1] * W + kOff3[c][0]];
    }
    T off = (T)0;
#pragma unroll
    for (int c = 1; c < 15; ++c) off += cq[c] * nb[c];
    return off;
  };
  // pair slot t: LDS row jj = 1 + t / 32 (the rows of the one-point halo region) and columns
  // (2 c, 2 c + 1), c = t % 32; the parity alternates along i, so one point of the pair is red
  // and the other black.  The red phase takes the pairs' red points in the halo region
  // (columns 1 .. W - 2), the black phase the pairs of the tile (rows 2 .. H - 3, c = 1 .. 30)
  auto pair_pts = [&](int t, int q, int& jj, int& ir, int& ib) {
    jj = 1 + (t >> 5);
    const int c2 = 2 * (t & 31);
    const int cl = col(i0 - 2 + c2, j0 - 2 + jj, q);
    ir = c2 + cl;
    ib = c2 + 1 - cl;
  };
  auto tile_pair = [&](int t) { const int jj = 1 + (t >> 5), c = t & 31; return jj >= 2 && jj < H - 2 && c >= 1 && c < W / 2 - 1; };
  // global loads run ahead: u of plane p + 1, and b of plane p at both points of every pair,
  // are in flight while plane p is processed (the barriers wait for LDS only); b of the red
  // points is used one plane later, b of the black points two.  Points outside the closure (or
  // outside the interior, for b) load offset 0 and are then replaced by zero
  T ureg[NP], bR[RQ], bRn[RQ], bB[RQ], bB1[RQ], bBn[RQ];
  auto ld = [&](const __amdgpu_buffer_rsrc_t& r, bool ok, int i, int j, int k) {
    T v;
    d_bload(r, ok ? (uint32_t)(plane(k) + rowin(j, k) + i) * (uint32_t)sizeof(T) : 0u, v);
    return ok ? v : (T)0;
  };
  auto load_u = [&](int p) {
#pragma unroll
    for (int s = 0; s < NP; ++s) {
      const int i = i0 - 2 + lane, j = j0 - 2 + w4 + 4 * s;
      ureg[s] = ld(ru, p >= 0 && i >= 0 && j >= 0 && i + j + p <= n, i, j, p);
    }
  };
  auto load_b = [&](int q) {
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
      const int t = tid + 256 * r;
      int jj = 1, ir = 1, ib = 2;
      if (t < NQ) pair_pts(t, q, jj, ir, ib);
      const int j = j0 - 2 + jj;
      const bool qr = t < NQ && q >= k0 - 1 && q <= k1 && ir >= 1 && ir < W - 1;
      const bool qbk = t < NQ && q >= k0 && q < k1 && tile_pair(t);
      bRn[r] = ld(rb, qr && inner(i0 - 2 + ir, j, q), i0 - 2 + ir, j, q);
      bBn[r] = ld(rb, qbk && inner(i0 - 2 + ib, j, q), i0 - 2 + ib, j, q);
    }
  };
#pragma unroll
  for (int r = 0; r < RQ; ++r) bR[r] = bRn[r] = bB[r] = bB1[r] = bBn[r] = (T)0;
  load_u(k0 - 2);
  for (int p = k0 - 2; p <= k1 + 1; ++p) {
    {
      T* U = sU[slot(p)];
#pragma unroll
      for (int s = 0; s < NP; ++s) U[(w4 + 4 * s) * W + lane] = ureg[s];
    }
    if (p + 1 <= k1 + 1) load_u(p + 1);
    load_b(p);
    __syncthreads();
    const int q = p - 1;   // red points of plane q on the tile and the one-point halo, in place
    if (q >= k0 - 1 && q <= k1) {
      const T* Um = sU[slot(q - 1)];
      T* U0 = sU[slot(q)];
      const T* Up = sU[slot(q + 1)];
#pragma unroll
      for (int r = 0; r < RQ; ++r) {
        const int t = tid + 256 * r;
        if (t >= NQ) continue;
        int jj, ir, ib;
        pair_pts(t, q, jj, ir, ib);
        if (ir < 1 || ir >= W - 1 || !inner(i0 - 2 + ir, j0 - 2 + jj, q)) continue;
        const int idx = jj * W + ir;
        const T off = stencil(Um, U0, Up, idx);
        U0[idx] = (bR[r] - off) / diag;
      }
    }
    __syncthreads();
    const int qb = p - 2;   // black points of plane qb on the tile; both colours written
    if (qb >= k0 && qb < k1) {
      const T* Rm = sU[slot(qb - 1)];
      const T* R0 = sU[slot(qb)];
      const T* Rp = sU[slot(qb + 1)];
      const int pk = plane(qb);
#pragma unroll
      for (int r = 0; r < RQ; ++r) {
        const int t = tid + 256 * r;
        if (t >= NQ || !tile_pair(t)) continue;
        int jj, ir, ib;
        pair_pts(t, qb, jj, ir, ib);
        const int j = j0 - 2 + jj, gi = i0 - 2 + ib, gr = i0 - 2 + ir;
        const int row = pk + rowin(j, qb);
        if (inner(gi, j, qb)) {
          const T off = stencil(Rm, R0, Rp, jj * W + ib);
          d_bstore(ro, (uint32_t)(row + gi) * (uint32_t)sizeof(T), (bB[r] - off) / diag);
        }
        if (inner(gr, j, qb)) d_bstore(ro, (uint32_t)(row + gr) * (uint32_t)sizeof(T), R0[jj * W + ir]);
      }
    }
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
      bR[r] = bRn[r];
      bB[r] = bB1[r];
      bB1[r] = bBn[r];
    }
  }
}

// Red-black Gauss-Seidel sweep of all macro interiors of a 3D level with n <= NMAX (NMAX <= 65),
// both colours in one launch, out of place: reads u, writes the interior of uo and copies the
// interface points of u into uo (so uo holds the whole iterate after the launch).  One workgroup
// streams the planes k0 .. k1-1 of one macro.  A plane of the closure (the points of height k,
// a triangle of side n - k stored contiguously) is copied whole into LDS, so in-plane
// neighbours need no halo and the copy is one contiguous run.  Per plane p: copy plane p, update
// the red points of plane p-1 in place in LDS (red points read only black neighbours), then the
// black points of plane p-2, and write both colours of plane p-2.  The red points of the planes
// k0-1 and k1 are recomputed from old values, identically to the workgroup that owns them.
// A wavefront takes a pair of interior rows j and R+1-j of a plane (R rows): their lengths add
// up to n-1-k, so the pair fills the lanes of one wavefront about evenly over the triangle.
// Loads run two planes ahead: u of plane p+2 and b of plane p+1 are in flight while plane p is
// processed (the step loop is unrolled by four so that every register set is fixed).  Same
// updates, in the same order within each point, as the class-by-class sweep: red (parity 0)
// first, then black; interface points are left to the interface sweep.
template <typename T, int NMAX, bool FINE>
__global__ void __launch_bounds__(512) k_gs3d_planes(LK lk, Tables tb, const T* __restrict__ u, T* __restrict__ uo,
                                                     const T* __restrict__ b, const int32_t* __restrict__ chunks,
                                                     int nchunks, double sA) {
  constexpr int NW = 8, NS = 5;
  constexpr int PS = (NMAX + 1) * (NMAX + 2) / 2;   // the largest plane (k = 0)
  constexpr int NL = (PS + 511) / 512;
  constexpr int RU = ((NMAX - 2) / 2 + NW - 1) / NW;   // row pairs per wavefront
  static_assert(NMAX <= 65, "a row pair must fit one wavefront");
  __shared__ T sU[NS * PS];
  const int per_xcd = (int)(gridDim.x >> 3);   // gridDim.x is a multiple of 8
  const int blk = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  if (blk >= lk.nmacro * nchunks) return;
  const int m = blk / nchunks;
  const int ch = chunks[blk - m * nchunks];
  const int k0 = ch & 0xffff, k1 = ch >> 16;   // interior planes k0 .. k1-1 (1 <= k0 < k1 <= n - 2)
  const int n = lk.n;
  const int64_t base = (int64_t)m * lk.S;
  const uint32_t mbytes = (uint32_t)(lk.S * (int64_t)sizeof(T));
  const __amdgpu_buffer_rsrc_t ru = d_rsrc(u + base, mbytes), rbr = d_rsrc(b + base, mbytes),
                               ro = d_rsrc(uo + base, mbytes);
  const double* Wt = tb.stiff + (size_t)m * kMaxMask * 15;
  const double ks = sA * tb.kappa[m];
  const T diag = (T)(ks * Wt[0]);
  T cq[15];
#pragma unroll
  for (int q = 1; q < 15; ++q) cq[q] = (T)(ks * Wt[q]);
  const int* rp = tb.rbpar + m * 4;
  const int s1 = rp[1], s2 = rp[2], s3 = rp[3];
  const int tid = (int)threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int dn = d_tet(n);
  auto plane = [&](int k) { return dn - d_tet(n - k); };                       // first point of plane k
  auto psize = [&](int k) { return ((n - k + 1) * (n - k + 2)) >> 1; };
  auto rowin = [&](int j, int k) { return j * (n - k + 1) - ((j * (j - 1)) >> 1); };   // row j within plane k
  auto slot = [](int k) { return ((k + NS) % NS) * PS; };
  // interior point (i, row) of this lane in row pair r of plane q; false if the lane idles
  auto lanept = [&](int q, int r, int& row, int& i) {
    const int pr = w + NW * r;
    const int j = 1 + pr, j2 = n - 2 - q - pr;   // rows j and R + 1 - j, R = n - 2 - q
    const int len1 = n - 1 - q - j, len2 = j2 > j ? j : 0;
    const bool first = lane < len1;
    row = first ? j : j2;
    i = first ? lane + 1 : lane - len1 + 1;
    return j <= j2 && lane < len1 + len2;
  };
  T U[2][NL], B[4][RU];
  // loads past the end of a plane (or of the needed rows) take distinct offsets outside the
  // buffer and return zero: no select on (or copy of) a loaded value, which would wait for it
  constexpr uint32_t kOut = 0xFFFFFFF0u;
  auto load_u = [&](T (&reg)[NL], int p) {
    const int sz = p >= 0 && p <= n ? psize(p) : 0;
    const uint32_t o0 = p >= 0 ? (uint32_t)plane(p) : 0u;
#pragma unroll
    for (int s = 0; s < NL; ++s) {
      const int t = tid + 512 * s;
      d_bload(ru, t < sz ? (o0 + (uint32_t)t) * (uint32_t)sizeof(T) : kOut - 64u * s, reg[s]);
    }
  };
  // b at this lane's interior points of plane p (loaded one step ahead: used by the red update
  // two steps later, by the black update three steps later)
  auto load_b = [&](T (&reg)[RU], int p) {
    const bool need = p >= k0 - 1 && p <= k1 && p >= 1;
#pragma unroll
    for (int r = 0; r < RU; ++r) {
      int row, i;
      const bool ok = need && lanept(p, r, row, i);
      d_bload(rbr, ok ? (uint32_t)(plane(p) + rowin(row, p) + i) * (uint32_t)sizeof(T) : kOut - 64u * r, reg[r]);
    }
  };
  // off-diagonal part of the row of interior point (i, row, q) from the LDS planes q-1, q, q+1,
  // r00 = rowin(row, q).  The 14 neighbours lie on 7 rows (row + b of plane q + c); their
  // offsets follow from r00 by additions: rowin(r + 1, k) = rowin(r, k) + (n - k + 1) - r and
  // rowin(r, k + 1) = rowin(r, k) - r
  auto stencil = [&](int row, int i, int q, int r00) {
    const int n1 = n - q + 1, s0 = slot(q), sp = slot(q + 1), sm = slot(q - 1);
    const int c00 = s0 + r00 + i, cp0 = c00 + n1 - row, cm0 = c00 - n1 + row - 1;
    const int c0p = sp + r00 + i - row, c0m = sm + r00 + i + row;
    const int cmp = sp + r00 + i - n1, cpm = sm + r00 + i + n1 + 1;
    T off = (T)0;
#pragma unroll
    for (int c = 1; c < 15; ++c) {
      const int bb = kOff3[c][1], kc = kOff3[c][2];
      const int at = kc == 0 ? (bb == 0 ? c00 : (bb > 0 ? cp0 : cm0))
                             : (kc > 0 ? (bb == 0 ? c0p : cmp) : (bb == 0 ? c0m : cpm));
      off += cq[c] * sU[at + kOff3[c][0]];
    }
    return off;
  };
  const int p0 = k0 - 2;
  // the apex (plane n, one point) is copied by the last chunk
  if (k1 == n - 2 && tid == 0) {
    T v;
    d_bload(ru, (uint32_t)plane(n) * (uint32_t)sizeof(T), v);
    d_bstore(ro, (uint32_t)plane(n) * (uint32_t)sizeof(T), v);
  }
  load_u(U[0], p0);
  load_u(U[1], p0 + 1);
  load_b(B[0], p0);
  for (int pb = p0; pb <= k1 + 1; pb += 4) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int p = pb + s;
      if (p > k1 + 1) break;
      if (p >= 0) {
        const int sz = psize(p);
        T* Sl = sU + slot(p);
#pragma unroll
        for (int e = 0; e < NL; ++e) {
          const int t = tid + 512 * e;
          if (t < sz) Sl[t] = U[s & 1][e];
        }
      }
      if (p + 2 <= k1 + 1) load_u(U[s & 1], p + 2);
      if (p + 1 <= k1) load_b(B[(s + 1) & 3], p + 1);   // the set of plane p - 3, no longer read
      __syncthreads();
      // the interface points of plane p (the macro boundary: i = 0, j = 0 or i + j = n - p, and
      // all of plane 0), which the sweep does not change, go from LDS into uo as well, so that
      // the interface classes can update uo in place.  Each plane is copied by one workgroup:
      // the planes of its chunk, plane 0 by the first chunk, planes n-2 and n-1 by the last
      if (p >= 0 && ((p >= k0 && p < k1) || (k0 == 1 && p == 0) || (k1 == n - 2 && p >= n - 2))) {
        const int mm = n - p, nb = p == 0 ? psize(0) : 3 * mm, pp = plane(p);
        const T* Sl = sU + slot(p);
        for (int t = tid; t < nb; t += 512) {
          int li = t;   // plane 0: every point, in order
          if (p > 0) {
            int i, j;
            if (t <= mm) { i = t; j = 0; }
            else if (t <= 2 * mm) { i = 0; j = t - mm; }
            else { j = t - 2 * mm; i = mm - j; }
            li = rowin(j, p) + i;
          }
          d_bstore(ro, (uint32_t)(pp + li) * (uint32_t)sizeof(T), Sl[li]);
        }
      }
      const int q = p - 1;   // red points of plane q, in place (b of plane q: set s + 3)
      if (q >= k0 - 1 && q <= k1 && q >= 1) {
#pragma unroll
        for (int r = 0; r < RU; ++r) {
          int row, i;
          if (lanept(q, r, row, i) && ((i * s1 + row * s2 + q * s3) & 1) == 0) {
            const int r00 = rowin(row, q);
            const T off = stencil(row, i, q, r00);
            sU[slot(q) + r00 + i] = (B[(s + 3) & 3][r] - off) / diag;
          }
        }
      }
      __syncthreads();
      const int qb = p - 2;   // black points of plane qb (b: set s + 2); both colours written
      if (qb >= k0 && qb < k1) {
        const int pk = plane(qb);
#pragma unroll
        for (int r = 0; r < RU; ++r) {
          int row, i;
          if (lanept(qb, r, row, i)) {
            const int r00 = rowin(row, qb), li = r00 + i;
            T v;
            if ((i * s1 + row * s2 + qb * s3) & 1) v = (B[(s + 2) & 3][r] - stencil(row, i, qb, r00)) / diag;
            else v = sU[slot(qb) + li];
            d_bstore(ro, (uint32_t)(pk + li) * (uint32_t)sizeof(T), v);
          }
        }
      }
    }
  }
}

// Gauss-Seidel (or Jacobi) update of one interface DoF t: the assembled row is the sum of the
// partial rows of all macros containing it.  Interior neighbours are read from xi, interface
// neighbours (and the DoF's own old value) from xf; the new value goes to every copy in uout
// and, if given, in umirror.  (xi and xf differ during the out-of-place 2D sweep.)
template <int D, typename T, bool P1>
__device__ __forceinline__ void iface_update(const LK& lk, const Tables& tb, int64_t t, const T* xi, const T* xf, T* uout,
                                             T* umirror, const T* __restrict__ b, int jacobi, double omega, double sA,
                                             const double* __restrict__ kn) {
  constexpr int NV = D + 1;
  int p, co[3], np;
  d_iface_decode(lk, tb, t, p, co, np);
  const int q0 = tb.inc_off[p], q1 = tb.inc_off[p + 1];
  const bool dir = tb.primdir[p] != 0;
  T rhs = (T)0, off = (T)0, diag = (T)0, uold = (T)0;
  for (int q = q0; q < q1; ++q) {
    const Inc in = tb.inc[q];
    int lc[4] = {0, 0, 0, 0};
    for (int r = 0; r < np; ++r) lc[in.slot[r]] = co[r];
    const int i = lc[1], j = lc[2], k = lc[3];
    const int64_t base = (int64_t)in.macro * lk.S;
    const int ctr = d_lin<D>(lk.n, i, j, k);
    if (q == q0) uold = xf[base + ctr];
    if (dir) continue;
    rhs += b[base + ctr];
    if constexpr (P1) {
      const double* EK = tb.elemK + (size_t)in.macro * ntype<D>() * NV * NV;
      const uint32_t iv = tb.incvalid[in.mask];
      for (int ty = 0; ty < ntype<D>(); ++ty) {
        for (int a = 0; a < NV; ++a) {
          if (!((iv >> (ty * NV + a)) & 1)) continue;
          int oa0, oa1, oa2;
          d_typeoff<D>(ty, a, oa0, oa1, oa2);
          T val[NV];
          double ks = 0.0;
          for (int bb = 0; bb < NV; ++bb) {
            int o0, o1, o2;
            d_typeoff<D>(ty, bb, o0, o1, o2);
            const int i2 = i + o0 - oa0, j2 = j + o1 - oa1, k2 = k + o2 - oa2;
            const int l2 = d_lin<D>(lk.n, i2, j2, k2);
            val[bb] = (d_mask<D>(lk.n, i2, j2, k2) ? xf : xi)[base + l2];
            ks += kn[base + l2];
          }
          ks *= sA / NV;
          const double* Kr = EK + (ty * NV + a) * NV;
          for (int bb = 0; bb < NV; ++bb) {
            if (bb == a) diag += (T)(ks * Kr[bb]);
            else off += (T)(ks * Kr[bb]) * val[bb];
          }
        }
      }
    } else {
      const double* W = tb.stiff + ((size_t)in.macro * kMaxMask + in.mask) * ndir<D>();
      const uint32_t valid = tb.validdirs[in.mask];
      const double scale = sA * tb.kappa[in.macro];
      const NbrIdx<D> nb(lk.n, i, j, k);
#pragma unroll
      for (int dd = 1; dd < ndir<D>(); ++dd) {
        if (!((valid >> dd) & 1)) continue;
        int a, b2, c;
        d_off<D>(dd, a, b2, c);
        const int i2 = i + a, j2 = j + b2, k2 = k + c;
        off += (T)(scale * W[dd]) * (d_mask<D>(lk.n, i2, j2, k2) ? xf : xi)[base + nb.at(dd)];
      }
      diag += (T)(scale * W[0]);
    }
  }
  T unew;
  if (dir) unew = uold;
  else if (jacobi) unew = uold + (T)omega * (rhs - off - diag * uold) / diag;
  else unew = (rhs - off) / diag;
  for (int q = q0; q < q1; ++q) {
    const Inc in = tb.inc[q];
    int lc[4] = {0, 0, 0, 0};
    for (int r = 0; r < np; ++r) lc[in.slot[r]] = co[r];
    const int64_t ix = (int64_t)in.macro * lk.S + d_lin<D>(lk.n, lc[1], lc[2], lc[3]);
    uout[ix] = unew;
    if (umirror) umirror[ix] = unew;
  }
}

template <int D, typename T, bool P1>
__global__ void __launch_bounds__(256) k_smooth_iface(LK lk, Tables tb, const int32_t* __restrict__ list, int count,
                                                       const T* xi, const T* xf, T* uout, T* umirror,
                                                       const T* __restrict__ b, int jacobi, double omega, double sA,
                                                       const double* __restrict__ kn) {
  const int tid = blockIdx.x * 256 + threadIdx.x;
  if (tid >= count) return;
  iface_update<D, T, P1>(lk, tb, list ? (int64_t)list[tid] : (int64_t)tid, xi, xf, uout, umirror, b, jacobi, omega, sA,
                         kn);
}

// every interface colour class c0..c1-1 of one sweep in a single workgroup (small levels):
// one launch instead of one per class, classes separated by barriers
template <int D, typename T, bool P1>
__global__ void __launch_bounds__(1024) k_iface_sweep_1wg(LK lk, Tables tb, const int32_t* __restrict__ list,
                                                           const int32_t* __restrict__ coff, int c0, int c1,
                                                           const T* xi, const T* xf, T* uout, T* umirror,
                                                           const T* __restrict__ b, double sA,
                                                           const double* __restrict__ kn) {
  for (int c = c0; c < c1; ++c) {
    const int e = coff[c + 1];
    for (int k = coff[c] + (int)threadIdx.x; k < e; k += (int)blockDim.x)
      iface_update<D, T, P1>(lk, tb, (int64_t)list[k], xi, xf, uout, umirror, b, 0, 0.0, sA, kn);
    __syncthreads();
  }
}

// Lane-parallel interface update: one lane per (interface DoF, incident macro) pair, the lanes
// of one DoF consecutive inside a wavefront (a segment).  Each lane computes its macro's
// partial row (right-hand side, off-diagonal sum, diagonal) from the copy's closure
// neighbours; every lane of a segment then sums the segment's partials in the same order
// through lane shuffles, so all copies receive bitwise the same new value, which each lane
// writes to its own copy.  A lane's task gives its copy's level-vector index, macro, zero-set
// mask and closure coordinates directly, so the update is one table load and one gather,
// whatever the number of copies.  Level vectors are accessed through buffer descriptors
// bounded to the level (nfull entries).  wmax[w]: longest segment of wavefront w.
template <int D, typename T>
__device__ __forceinline__ void iface_task_wave(const LK& lk, const Tables& tb, const int32_t* __restrict__ tcopy,
                                                const int32_t* __restrict__ tinfo, const int32_t* __restrict__ tloc,
                                                const int32_t* __restrict__ tseg, int wmax, int w, const T* xi,
                                                const T* xf, T* uout, T* umirror, const T* __restrict__ b, int jacobi,
                                                double omega, double sA) {
  const int lane = threadIdx.x & 63;
  const int idx = w * 64 + lane;
  const uint32_t vbytes = (uint32_t)((int64_t)lk.nmacro * lk.S) * (uint32_t)sizeof(T);
  const __amdgpu_buffer_rsrc_t rxi = d_rsrc(xi, vbytes), rxf = d_rsrc(xf, vbytes), rb = d_rsrc(b, vbytes);
  const bool same = xi == xf;
  const int cp = tcopy[idx];
  const int info = tinfo[idx], loc = tloc[idx], seg = tseg[idx];
  T rhs = (T)0, off = (T)0, diag = (T)0, uold = (T)0;
  const bool live = cp >= 0;
  const bool dir = (info >> 28) & 1;
  if (live) {
    const int m = info & 0xffffff, mask = (info >> 24) & 15;
    const int i = loc & 2047, j = (loc >> 11) & 2047, k = loc >> 22;
    const int64_t base = (int64_t)m * lk.S;
    d_bload(rxf, (uint32_t)cp * (uint32_t)sizeof(T), uold);
    if (!dir) {
      d_bload(rb, (uint32_t)cp * (uint32_t)sizeof(T), rhs);
      const double* W = tb.stiff + ((size_t)m * kMaxMask + mask) * ndir<D>();
      const uint32_t valid = tb.validdirs[mask];
      const double scale = sA * tb.kappa[m];
      const NbrIdx<D> nb(lk.n, i, j, k);
#pragma unroll
      for (int dd = 1; dd < ndir<D>(); ++dd) {
        if (!((valid >> dd) & 1)) continue;
        int a, b2, c;
        d_off<D>(dd, a, b2, c);
        const int i2 = i + a, j2 = j + b2, k2 = k + c;
        const uint32_t li = (uint32_t)(base + nb.at(dd));
        const uint32_t o = li * (uint32_t)sizeof(T);
        T v;
        if (same) {
          d_bload(rxf, o, v);
        } else {
          // interface neighbours from xf, interior ones from xi: one load through a per-lane
          // address (a buffer descriptor must be wave-uniform)
          v = (d_mask<D>(lk.n, i2, j2, k2) ? xf : xi)[li];
        }
        off += (T)(scale * W[dd]) * v;
      }
      diag = (T)(scale * W[0]);
    }
  }
  // segment sums of (rhs - off) and diag; every lane of the wavefront takes part in every
  // shuffle
  const int lead = seg & 63, len = seg >> 8;
  const T num = rhs - off;
  T snum = (T)0, sdiag = (T)0;
  for (int kq = 0; kq < wmax; ++kq) {
    const int src = min(lead + kq, 63);
    const T a = __shfl(num, src, 64), d = __shfl(diag, src, 64);
    if (kq < len) { snum += a; sdiag += d; }
  }
  if (!live) return;
  T unew;
  if (dir) unew = uold;
  else if (jacobi) unew = uold + (T)omega * (snum - sdiag * uold) / sdiag;
  else unew = snum / sdiag;
  const uint32_t oc = (uint32_t)cp * (uint32_t)sizeof(T);
  d_bstore(d_rsrc(uout, vbytes), oc, unew);
  if (umirror) d_bstore(d_rsrc(umirror, vbytes), oc, unew);
}

// one interface colour class: wavefronts w0 .. w1-1, four per block
template <int D, typename T>
__global__ void __launch_bounds__(256) k_iface_tasks(LK lk, Tables tb, const int32_t* __restrict__ tcopy,
                                                      const int32_t* __restrict__ tinfo, const int32_t* __restrict__ tloc,
                                                      const int32_t* __restrict__ tseg, const int32_t* __restrict__ wmax,
                                                      int w0, int w1, const T* xi, const T* xf, T* uout, T* umirror,
                                                      const T* __restrict__ b, int jacobi, double omega, double sA) {
  const int w = __builtin_amdgcn_readfirstlane(w0 + d_xcd_block() * 4 + (int)(threadIdx.x >> 6));
  if (w >= w1) return;
  iface_task_wave<D, T>(lk, tb, tcopy, tinfo, tloc, tseg, wmax[w], w, xi, xf, uout, umirror, b, jacobi, omega, sA);
}

// every interface class c0..c1-1 of one sweep in one workgroup of 16 wavefronts (small
// levels), classes separated by barriers; woff[c] is the first wavefront of class c
template <int D, typename T>
__global__ void __launch_bounds__(1024) k_iface_tasks_1wg(LK lk, Tables tb, const int32_t* __restrict__ tcopy,
                                                           const int32_t* __restrict__ tinfo, const int32_t* __restrict__ tloc,
                                                           const int32_t* __restrict__ tseg,
                                                           const int32_t* __restrict__ wmax,
                                                           const int32_t* __restrict__ woff, int c0, int c1, const T* xi,
                                                           const T* xf, T* uout, T* umirror, const T* __restrict__ b,
                                                           double sA, int sweeps) {
  const int wave = (int)(threadIdx.x >> 6);
  for (int sw = 0; sw < sweeps; ++sw)
    for (int c = c0; c < c1; ++c) {
      const int e = woff[c + 1];
      for (int w = woff[c] + wave; w < e; w += 16)
        iface_task_wave<D, T>(lk, tb, tcopy, tinfo, tloc, tseg, wmax[w], w, xi, xf, uout, umirror, b, 0, 0.0, sA);
      __syncthreads();
    }
}

// The same classes in one workgroup with the sweep-invariant part of every row loaded before
// the first class: task records, right-hand side, stencil weights, and the values of interior
// neighbours (final once the macro interiors are swept).  Each class then reloads only its
// interface neighbours, so a class costs one dependent memory round trip instead of two.
// Wave v takes wavefront woff[c] + v of class c0 + k for k < P (the host launches this form
// only when every class has at most 16 wavefronts and c1 - c0 <= P).  Rows are summed in the
// same order as iface_task_wave, so both forms give identical results.
template <int D, typename T>
struct TaskPre {
  int cp, seg, wmax, info;
  uint32_t valid, ifm;
  T rhs, diag, uold;
  T coef[ndir<D>() - 1], v[ndir<D>() - 1];
  uint32_t o[ndir<D>() - 1];
};

template <int D, typename T>
__device__ __forceinline__ void task_pre_load(const LK& lk, const Tables& tb, const int32_t* __restrict__ tcopy,
                                              const int32_t* __restrict__ tinfo, const int32_t* __restrict__ tloc,
                                              const int32_t* __restrict__ tseg, int w,
                                              const __amdgpu_buffer_rsrc_t& rxi, const __amdgpu_buffer_rsrc_t& rxf,
                                              const __amdgpu_buffer_rsrc_t& rb, double sA, TaskPre<D, T>& q) {
  const int idx = w * 64 + (int)(threadIdx.x & 63);
  q.cp = tcopy[idx];
  q.info = tinfo[idx];
  q.seg = tseg[idx];
  const int loc = tloc[idx];
  q.valid = 0;
  q.ifm = 0;
  q.rhs = (T)0;
  q.diag = (T)0;
  q.uold = (T)0;
#pragma unroll
  for (int dd = 0; dd < ndir<D>() - 1; ++dd) { q.coef[dd] = (T)0; q.v[dd] = (T)0; q.o[dd] = 0; }
  if (q.cp < 0) return;
  const bool dir = (q.info >> 28) & 1;
  const int m = q.info & 0xffffff, mask = (q.info >> 24) & 15;
  const int i = loc & 2047, j = (loc >> 11) & 2047, k = loc >> 22;
  const int64_t base = (int64_t)m * lk.S;
  d_bload(rxf, (uint32_t)q.cp * (uint32_t)sizeof(T), q.uold);
  if (dir) return;
  d_bload(rb, (uint32_t)q.cp * (uint32_t)sizeof(T), q.rhs);
  const double* W = tb.stiff + ((size_t)m * kMaxMask + mask) * ndir<D>();
  q.valid = tb.validdirs[mask];
  const double scale = sA * tb.kappa[m];
  const NbrIdx<D> nb(lk.n, i, j, k);
#pragma unroll
  for (int dd = 1; dd < ndir<D>(); ++dd) {
    if (!((q.valid >> dd) & 1)) continue;
    int a, b2, c;
    d_off<D>(dd, a, b2, c);
    const int i2 = i + a, j2 = j + b2, k2 = k + c;
    q.o[dd - 1] = (uint32_t)(base + nb.at(dd)) * (uint32_t)sizeof(T);
    q.coef[dd - 1] = (T)(scale * W[dd]);
    if (d_mask<D>(lk.n, i2, j2, k2)) q.ifm |= 1u << dd;
    else d_bload(rxi, q.o[dd - 1], q.v[dd - 1]);
  }
  q.diag = (T)(scale * W[0]);
}

template <int D, typename T>
__device__ __forceinline__ void task_pre_finish(const __amdgpu_buffer_rsrc_t& rxf, TaskPre<D, T>& q, T* uout,
                                                T* umirror, uint32_t vbytes) {
  const bool live = q.cp >= 0;
  const bool dir = (q.info >> 28) & 1;
  T off = (T)0;
  if (live && !dir) {
#pragma unroll
    for (int dd = 1; dd < ndir<D>(); ++dd) {
      if (!((q.valid >> dd) & 1)) continue;
      if ((q.ifm >> dd) & 1) d_bload(rxf, q.o[dd - 1], q.v[dd - 1]);
      off += q.coef[dd - 1] * q.v[dd - 1];
    }
  }
  const int lead = q.seg & 63, len = q.seg >> 8;
  const T num = q.rhs - off, diag = q.diag;
  T snum = (T)0, sdiag = (T)0;
  for (int kq = 0; kq < q.wmax; ++kq) {
    const int src = min(lead + kq, 63);
    const T a = __shfl(num, src, 64), d = __shfl(diag, src, 64);
    if (kq < len) { snum += a; sdiag += d; }
  }
  if (!live) return;
  const T unew = dir ? q.uold : snum / sdiag;
  const uint32_t oc = (uint32_t)q.cp * (uint32_t)sizeof(T);
  d_bstore(d_rsrc(uout, vbytes), oc, unew);
  if (umirror) d_bstore(d_rsrc(umirror, vbytes), oc, unew);
}

// classes held in registers at once within the register budget of a 1024-thread workgroup:
// four float rows in 2D, two double rows in 2D or float rows in 3D; double rows in 3D (14
// neighbours) do not fit and use the plain form
template <int D, typename T>
constexpr int pre_classes() { return D == 2 ? (sizeof(T) == 4 ? 4 : 2) : (sizeof(T) == 4 ? 2 : 0); }

int iface_pre_classes(int dim, bool dbl) {
  return dim == 2 ? (dbl ? pre_classes<2, double>() : pre_classes<2, float>())
                  : (dbl ? pre_classes<3, double>() : pre_classes<3, float>());
}

template <int D, typename T, int P>
__global__ void __launch_bounds__(1024) k_iface_tasks_1wg_pre(LK lk, Tables tb, const int32_t* __restrict__ tcopy,
                                                               const int32_t* __restrict__ tinfo,
                                                               const int32_t* __restrict__ tloc,
                                                               const int32_t* __restrict__ tseg,
                                                               const int32_t* __restrict__ wmax,
                                                               const int32_t* __restrict__ woff, int c0, int c1,
                                                               const T* xi, const T* xf, T* uout, T* umirror,
                                                               const T* __restrict__ b, double sA) {
  const int wave = (int)(threadIdx.x >> 6);
  const uint32_t vbytes = (uint32_t)((int64_t)lk.nmacro * lk.S) * (uint32_t)sizeof(T);
  const __amdgpu_buffer_rsrc_t rxi = d_rsrc(xi, vbytes), rxf = d_rsrc(xf, vbytes), rb = d_rsrc(b, vbytes);
  TaskPre<D, T> q[P];
  bool has[P];
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const int c = c0 + k;
    const int w = c < c1 ? __builtin_amdgcn_readfirstlane(woff[c] + wave) : 0;
    has[k] = c < c1 && w < woff[c + 1];
    q[k].wmax = has[k] ? wmax[w] : 0;
    if (has[k]) task_pre_load<D, T>(lk, tb, tcopy, tinfo, tloc, tseg, w, rxi, rxf, rb, sA, q[k]);
  }
#pragma unroll
  for (int k = 0; k < P; ++k) {
    if (k < c1 - c0) {
      if (has[k]) task_pre_finish<D, T>(rxf, q[k], uout, umirror, vbytes);
      __syncthreads();
    }
  }
}

// The two 2D edge classes of one level in one launch.  Wavefront v of workgroup g takes chunk
// v mod nch (64 consecutive points a = 1 + 64 c .. 64 c + 64) of edge g * epb + v / nch, so
// an edge's chunks sit in consecutive wavefronts of one workgroup.  Everything the edge needs
// (incident macros, their vertex slots and zero-set masks, coefficients and stencils) is one
// record of kEdgeRecWords words read by the scalar unit; the point addresses follow from a.
// On a Dirichlet edge the wavefront copies the fixed values into the output buffers.
// Otherwise it updates the class a even (2 <= a <= n - 2) from the loaded old values, hands
// the new values to the odd class through LDS (a workgroup barrier between the two), and
// updates the odd class; the points next to the vertices (a = 1, n - 1) keep their old
// values, they belong to the vertex classes that follow.  A point's row is the sum of the
// partial rows of its (at most two) incident macros, summed in the order of the lane-parallel
// class kernels (identical results).  The copies of the Dirichlet vertices (dvcopy) are
// copied into the output buffers on the side.
template <typename T>
__device__ __forceinline__ void iface2d_edges_body(int vblk, int nvblk, T* s_e0, const LK& lk,
                                                   const int32_t* __restrict__ erec, int nE, int nch, int epb,
                                                   const int32_t* __restrict__ dvcopy, int n_dv, const T* xi,
                                                   const T* xf, T* uout, T* umirror, const T* __restrict__ b,
                                                   double sA) {
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = (int)(threadIdx.x & 63);
  const int n = lk.n;
  const int e = vblk * epb + wave / nch, chunk = wave - (wave / nch) * nch;
  const bool has = wave < epb * nch && e < nE;
  const bool same = xi == xf;
  // per lane: position a on the edge, its copies k < ncp (closure index cp[k]); per copy the
  // partial row: right-hand side, diagonal, and per direction the weight, the neighbour value
  // and whether the neighbour is the edge point a - 1 or a + 1 (side -1 / +1)
  int a = 0, ncp = 0;
  bool dir = false, isE = false;
  int64_t cp[2] = {0, 0};
  T rhs[2] = {(T)0, (T)0}, dg[2] = {(T)0, (T)0};
  T coef[2][kNDir2 - 1], val[2][kNDir2 - 1];
  int side[2][kNDir2 - 1];
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int dd = 0; dd < kNDir2 - 1; ++dd) { coef[k][dd] = (T)0; val[k][dd] = (T)0; side[k][dd] = 0; }
  uint32_t vmask[2] = {0u, 0u};
  if (has) {
    const int32_t* R = erec + (size_t)e * kEdgeRecWords;
    // every word of the record the lanes use, read before any of it is used (the record always
    // has room for two copies), so the copies' words do not wait for the header
    const int hdr = R[0];
    int cmac[2], csl[2];
    uint32_t cval[2];
    double ckw[2][kNDir2 + 1];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int32_t* C = R + 2 + kEdgeCopyWords * k;
      cmac[k] = C[0];
      csl[k] = C[1];
      cval[k] = (uint32_t)C[18];
      const double* KW = reinterpret_cast<const double*>(C + 2);   // kappa, then the 7 weights
#pragma unroll
      for (int d = 0; d <= kNDir2; ++d) ckw[k][d] = KW[d];
    }
    // keep the loads here: without a use the compiler sinks each into the branch that needs it,
    // behind the header's round trip
    asm volatile("" ::"s"(hdr), "s"(cmac[0]), "s"(cmac[1]), "s"(csl[0]), "s"(csl[1]), "s"(cval[0]), "s"(cval[1]));
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int d = 0; d <= kNDir2; ++d) asm volatile("" ::"s"(ckw[k][d]));
    ncp = min(hdr & 3, 2);   // 1 or 2 (checked by the host)
    dir = (hdr >> 2) & 1;
    a = 1 + 64 * chunk + lane;
    if (a <= n - 1) {
      isE = !dir && a >= 2 && a <= n - 2;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        if (k >= ncp) break;
        const int macro = cmac[k], sl = csl[k];
        const int s0 = sl & 3, s1 = (sl >> 8) & 3, mask = (sl >> 16) & 15;
        int lc[3] = {0, 0, 0};
        lc[s0] = n - a;
        lc[s1] = a;
        const int i = lc[1], j = lc[2];
        const int64_t base = (int64_t)macro * lk.S;
        cp[k] = base + d_lin2(n, i, j);
        if (!isE) continue;
        rhs[k] = b[cp[k]];
        const double* KW = ckw[k];
        const uint32_t valid = cval[k];
        vmask[k] = valid;
        const double scale = sA * KW[0];
#pragma unroll
        for (int dd = 1; dd < kNDir2; ++dd) {
          if (!((valid >> dd) & 1)) continue;
          int o0, o1, o2;
          d_off<2>(dd, o0, o1, o2);
          const int i2 = i + o0, j2 = j + o1;
          const int m2 = d_mask<2>(n, i2, j2, 0);
          const int64_t ix = base + d_lin2(n, i2, j2);
          coef[k][dd - 1] = (T)(scale * KW[1 + dd]);
          val[k][dd - 1] = same ? xf[ix] : (m2 ? xf : xi)[ix];
          if (m2) {
            // a neighbour on the macro boundary lies on this edge (or is one of its vertices)
            const int cc[3] = {n - i2 - j2, i2, j2};
            const int a2 = cc[s1];
            side[k][dd - 1] = (a2 >= 1 && a2 <= n - 1) ? a2 - a : 0;
          }
        }
        dg[k] = (T)(scale * KW[1]);
      }
    }
  }
  auto update = [&]() -> T {
    T snum = (T)0, sdiag = (T)0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (k >= ncp) break;
      T off = (T)0;
#pragma unroll
      for (int dd = 1; dd < kNDir2; ++dd) {
        if (!((vmask[k] >> dd) & 1)) continue;
        off += coef[k][dd - 1] * val[k][dd - 1];
      }
      snum += rhs[k] - off;
      sdiag += dg[k];
    }
    return snum / sdiag;
  };
  auto store = [&](T v) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (k >= ncp) break;
      uout[cp[k]] = v;
      if (umirror) umirror[cp[k]] = v;
    }
  };
  const bool even = isE && (a & 1) == 0, odd = isE && (a & 1) == 1;
  T u = (T)0;
  if (even) {
    u = update();
    store(u);
  }
  s_e0[threadIdx.x + 1] = u;
  __syncthreads();
  if (odd) {
    // both edge neighbours are in the even class: their new values come from LDS (the
    // previous or next chunk of the edge sits in the neighbouring wavefront)
    const T um = s_e0[threadIdx.x], up = s_e0[threadIdx.x + 2];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int dd = 0; dd < kNDir2 - 1; ++dd) {
        if (side[k][dd] == -1) val[k][dd] = um;
        if (side[k][dd] == 1) val[k][dd] = up;
      }
    store(update());
  }
  if (dir && has && a <= n - 1) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (k >= ncp) break;
      const T v = xf[cp[k]];
      uout[cp[k]] = v;
      if (umirror) umirror[cp[k]] = v;
    }
  }
  const int bs = (int)blockDim.x;
  for (int q = vblk * bs + (int)threadIdx.x; q < n_dv; q += nvblk * bs) {
    const int c = dvcopy[q];
    const T v = xf[c];
    uout[c] = v;
    if (umirror) umirror[c] = v;
  }
}

template <typename T>
__global__ void __launch_bounds__(1024) k_iface2d_edges(LK lk, const int32_t* __restrict__ erec, int nE, int nch,
                                                         int epb, const int32_t* __restrict__ dvcopy, int n_dv,
                                                         const T* xi, const T* xf, T* uout, T* umirror,
                                                         const T* __restrict__ b, double sA) {
  __shared__ T s_e0[1024 + 2];
  iface2d_edges_body<T>((int)blockIdx.x, (int)gridDim.x, s_e0, lk, erec, nE, nch, epb, dvcopy, n_dv, xi, xf, uout,
                        umirror, b, sA);
}

template <typename T>
void launch_iface2d_edges(const LK& lk, const int32_t* erec, int nE, const int32_t* dvcopy, int n_dv, const T* xi,
                          const T* xf, T* uout, T* umirror, const T* b, double sA, hipStream_t st) {
  if (nE <= 0 && n_dv <= 0) return;
  const int nch = (lk.n - 1 + 63) / 64, epb = 16 / nch;
  const unsigned g = (unsigned)std::max(1, (nE + epb - 1) / epb);
  k_iface2d_edges<T><<<g, 1024, 0, st>>>(lk, erec, nE, nch, epb, dvcopy, n_dv, xi, xf, uout, umirror, b, sA);
}
template void launch_iface2d_edges<double>(const LK&, const int32_t*, int, const int32_t*, int, const double*,
                                           const double*, double*, double*, const double*, double, hipStream_t);
template void launch_iface2d_edges<float>(const LK&, const int32_t*, int, const int32_t*, int, const float*,
                                          const float*, float*, float*, const float*, double, hipStream_t);

// The 2D vertex classes of one level by wheels: a wheel is a macro vertex with the edge points
// next to it, and no point of one wheel touches another when n >= 4.  One lane per copy of
// each DoF of a wheel, the wheel's lanes inside one wavefront, its DoFs in class order.  Every
// lane loads its partial row once; then for each class in turn the lanes take the current
// values of same-wheel neighbours from the lanes holding them (new after their class, old
// before), the lanes of the class sum their partial rows over the copies of their DoF as the
// lane-parallel class kernel does (identical results), and keep the new value.  Neighbours
// outside the wheel (interior and edge-class points, already swept, and Dirichlet points)
// come from memory.
template <typename T>
__device__ __forceinline__ void iface2d_wheels_body(int w, const LK& lk, const Tables& tb,
                                                    const int32_t* __restrict__ wcopy,
                                                    const int32_t* __restrict__ winfo,
                                                    const int32_t* __restrict__ wloc,
                                                    const int32_t* __restrict__ wseg,
                                                    const int32_t* __restrict__ wsrc,
                                                    const double* __restrict__ wcw,
                                                    const int32_t* __restrict__ wwmax, int nwaves, int ncls,
                                                    const int32_t* __restrict__ we2, const int32_t* __restrict__ a2i,
                                                    const double* __restrict__ a2w, const T* xi, const T* xf, T* uout,
                                                    T* umirror,
                                                    const T* __restrict__ b, double sA) {
  if (w >= nwaves) return;
  const int n = lk.n;
  const int lane = (int)(threadIdx.x & 63);
  const int idx = w * 64 + lane;
  const int cp = wcopy[idx], info = winfo[idx], loc = wloc[idx], seg = wseg[idx];
  const uint32_t sa = (uint32_t)wsrc[2 * idx], sb = (uint32_t)wsrc[2 * idx + 1];
  const int wm = wwmax[w];
  const bool live = cp >= 0;
  const bool same = xi == xf;
  // the recompute tables of the one-launch form, loaded with the others (no dependence)
  int e2 = -1, ai[16];
  double aw[16];
  if (we2) {
    const int nl = nwaves * 64;
    e2 = we2[idx];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      ai[q] = a2i[(size_t)q * nl + idx];
      aw[q] = a2w[(size_t)q * nl + idx];
    }
  }
  T rhs = (T)0, dg = (T)0, u = (T)0;
  T coef[kNDir2 - 1], val[kNDir2 - 1];
#pragma unroll
  for (int dd = 0; dd < kNDir2 - 1; ++dd) { coef[dd] = (T)0; val[dd] = (T)0; }
  uint32_t valid = 0;
  int cls = -1;
  if (live) {
    const int m = info & 0xffffff, mask = (info >> 24) & 15;
    cls = (info >> 28) & 15;
    const int i = loc & 2047, j = loc >> 11;
    const int64_t base = (int64_t)m * lk.S;
    u = xf[cp];
    rhs = b[cp];
    // the lane's coefficient and unit stencil for its mask, one table entry per lane (struct
    // of arrays: kappa, then the 7 weights)
    const int nl = nwaves * 64;
    double W[kNDir2];
#pragma unroll
    for (int dd = 0; dd < kNDir2; ++dd) W[dd] = wcw[(size_t)(1 + dd) * nl + idx];
    valid = tb.validdirs[mask];
    const double scale = sA * wcw[idx];
#pragma unroll
    for (int dd = 1; dd < kNDir2; ++dd) {
      if (!((valid >> dd) & 1)) continue;
      int o0, o1, o2;
      d_off<2>(dd, o0, o1, o2);
      const int i2 = i + o0, j2 = j + o1;
      const int64_t ix = base + d_lin2(n, i2, j2);
      coef[dd - 1] = (T)(scale * W[dd]);
      val[dd - 1] = same ? xf[ix] : (d_mask<2>(n, i2, j2, 0) ? xf : xi)[ix];
    }
    dg = (T)(scale * W[0]);
    if (we2) {
      // the edge-class neighbour (a = 2 from the wheel's vertex) is swept in the same launch:
      // its new value is recomputed here from old values, with the same terms in the same order
      // as the edge classes compute it (bitwise the same).  Per lane and copy k of that point
      // (struct of arrays): a2i[8k] its closure index (-1: no such copy), a2i[8k + dd] the
      // neighbour in direction dd (-1: none), a2i[8k + 7] bit dd - 1 set if that neighbour is
      // an interface point (read from xf); a2w[8k] the macro's coefficient, a2w[8k + 1 + d] the
      // unit stencil weight d
      if (e2 >= 0) {
        const int dd2 = (e2 >> 25) & 7;
        T snum = (T)0, sdiag = (T)0;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int c2 = ai[8 * k];
          if (c2 < 0) break;
          const int fl = ai[8 * k + 7];
          const double sc = sA * aw[8 * k];
          const T r2 = b[c2];
          T off2 = (T)0;
#pragma unroll
          for (int dd = 1; dd < kNDir2; ++dd) {
            const int ix = ai[8 * k + dd];
            if (ix < 0) continue;
            const T v = ((fl >> (dd - 1)) & 1 ? xf : xi)[ix];
            off2 += (T)(sc * aw[8 * k + 1 + dd]) * v;
          }
          snum += r2 - off2;
          sdiag += (T)(sc * aw[8 * k + 1]);
        }
        const T v2 = snum / sdiag;
#pragma unroll
        for (int dd = 1; dd < kNDir2; ++dd)
          if (dd == dd2) val[dd - 1] = v2;
      }
    }
  }
  const int lead = seg & 63, len = seg >> 8;
  for (int c = 0; c < ncls; ++c) {
#pragma unroll
    for (int dd = 1; dd < kNDir2; ++dd) {
      const int s = (int)(((dd <= 4 ? sa >> (8 * (dd - 1)) : sb >> (8 * (dd - 5)))) & 0xffu);
      const T v = __shfl(u, s == 0xff ? lane : s, 64);
      if (s != 0xff) val[dd - 1] = v;
    }
    const bool mine = live && cls == c;
    T num = (T)0, diag = (T)0;
    if (mine) {
      T off = (T)0;
#pragma unroll
      for (int dd = 1; dd < kNDir2; ++dd) {
        if (!((valid >> dd) & 1)) continue;
        off += coef[dd - 1] * val[dd - 1];
      }
      num = rhs - off;
      diag = dg;
    }
    T snum = (T)0, sdiag = (T)0;
    for (int kq = 0; kq < wm; ++kq) {
      const int src = min(lead + kq, 63);
      const T a = __shfl(num, src, 64), d = __shfl(diag, src, 64);
      if (kq < len) { snum += a; sdiag += d; }
    }
    if (mine) u = snum / sdiag;
  }
  if (live) {
    uout[cp] = u;
    if (umirror) umirror[cp] = u;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_iface2d_wheels(LK lk, Tables tb, const int32_t* __restrict__ wcopy,
                                                         const int32_t* __restrict__ winfo,
                                                         const int32_t* __restrict__ wloc,
                                                         const int32_t* __restrict__ wseg,
                                                         const int32_t* __restrict__ wsrc,
                                                         const double* __restrict__ wcw,
                                                         const int32_t* __restrict__ wwmax, int nwaves, int ncls,
                                                         const T* xi, const T* xf, T* uout, T* umirror,
                                                         const T* __restrict__ b, double sA) {
  const int w = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + (int)(threadIdx.x >> 6));
  iface2d_wheels_body<T>(w, lk, tb, wcopy, winfo, wloc, wseg, wsrc, wcw, wwmax, nwaves, ncls, nullptr, nullptr, nullptr,
                         xi, xf, uout, umirror, b, sA);
}

// Both edge classes and all vertex classes of a 2D sweep in one launch (out of place, no
// mirror writes): workgroups 0 .. ge-1 sweep the edge classes as k_iface2d_edges does, the
// others the wheels (4 wavefronts each), which recompute their edge-class neighbours from
// per-lane tables instead of waiting for them.  Every value read is final before the launch
// (interior points in xi) or unchanged during it (xf), so the workgroups need no ordering; the
// result is bitwise that of the two launches.
template <typename T>
__global__ void __launch_bounds__(1024) k_iface2d_sweep(LK lk, Tables tb, const int32_t* __restrict__ erec, int nE,
                                                         int nch, int epb, int ge, const int32_t* __restrict__ dvcopy,
                                                         int n_dv, const int32_t* __restrict__ wcopy,
                                                         const int32_t* __restrict__ winfo,
                                                         const int32_t* __restrict__ wloc,
                                                         const int32_t* __restrict__ wseg,
                                                         const int32_t* __restrict__ wsrc,
                                                         const double* __restrict__ wcw,
                                                         const int32_t* __restrict__ wwmax, int nwaves, int ncls,
                                                         const int32_t* __restrict__ we2,
                                                         const int32_t* __restrict__ a2i,
                                                         const double* __restrict__ a2w, const T* xi, const T* xf,
                                                         T* uout, const T* __restrict__ b, double sA) {
  __shared__ T s_e0[1024 + 2];
  if ((int)blockIdx.x < ge) {
    iface2d_edges_body<T>((int)blockIdx.x, ge, s_e0, lk, erec, nE, nch, epb, dvcopy, n_dv, xi, xf, uout, nullptr, b,
                          sA);
    return;
  }
  // four wheel wavefronts per workgroup (the others idle): a wheel wavefront is a long chain of
  // shuffles and class steps, and more of them per compute unit only queue on its SIMDs
  const int wv = (int)(threadIdx.x >> 6);
  if (wv >= 4) return;
  const int w = __builtin_amdgcn_readfirstlane(((int)blockIdx.x - ge) * 4 + wv);
  iface2d_wheels_body<T>(w, lk, tb, wcopy, winfo, wloc, wseg, wsrc, wcw, wwmax, nwaves, ncls, we2, a2i, a2w, xi, xf,
                         uout, nullptr, b, sA);
}

template <typename T>
void launch_iface2d_sweep(const LK& lk, const Tables& tb, const int32_t* erec, int nE, const int32_t* dvcopy, int n_dv,
                          const int32_t* wcopy, const int32_t* winfo, const int32_t* wloc, const int32_t* wseg,
                          const int32_t* wsrc, const double* wcw, const int32_t* wwmax, int nwaves, int ncls,
                          const int32_t* we2, const int32_t* a2i, const double* a2w, const T* xi, const T* xf, T* uout,
                          const T* b, double sA, hipStream_t st) {
  // workgroups of 4 wavefronts while an edge fits them (n <= 257): the wheel workgroups then
  // carry no idle wavefronts and the edges are spread over more compute units; above that, one
  // edge per workgroup (the wheel part needs at least 4 wavefronts per workgroup)
  const int nch = (lk.n - 1 + 63) / 64, threads = nch <= 4 ? 256 : 64 * nch, epb = threads / 64 / nch;
  const int ge = std::max(1, (nE + epb - 1) / epb), gw = (nwaves + 3) / 4;
  k_iface2d_sweep<T><<<(unsigned)(ge + gw), (unsigned)threads, 0, st>>>(lk, tb, erec, nE, nch, epb, ge, dvcopy, n_dv,
                                                                        wcopy, winfo, wloc, wseg, wsrc, wcw, wwmax,
                                                                        nwaves, ncls, we2, a2i, a2w, xi, xf, uout, b,
                                                                        sA);
}
template void launch_iface2d_sweep<double>(const LK&, const Tables&, const int32_t*, int, const int32_t*, int,
                                           const int32_t*, const int32_t*, const int32_t*, const int32_t*,
                                           const int32_t*, const double*, const int32_t*, int, int, const int32_t*,
                                           const int32_t*, const double*, const double*, const double*, double*,
                                           const double*, double, hipStream_t);
template void launch_iface2d_sweep<float>(const LK&, const Tables&, const int32_t*, int, const int32_t*, int,
                                          const int32_t*, const int32_t*, const int32_t*, const int32_t*,
                                          const int32_t*, const double*, const int32_t*, int, int, const int32_t*,
                                          const int32_t*, const double*, const float*, const float*, float*,
                                          const float*, double, hipStream_t);

template <typename T>
void launch_iface2d_wheels(const LK& lk, const Tables& tb, const int32_t* wcopy, const int32_t* winfo,
                           const int32_t* wloc, const int32_t* wseg, const int32_t* wsrc, const double* wcw,
                           const int32_t* wwmax, int nwaves, int ncls, const T* xi, const T* xf, T* uout, T* umirror,
                           const T* b, double sA, hipStream_t st) {
  if (nwaves <= 0 || ncls <= 0) return;
  const unsigned g = (unsigned)((nwaves + 3) / 4);
  k_iface2d_wheels<T><<<g, 256, 0, st>>>(lk, tb, wcopy, winfo, wloc, wseg, wsrc, wcw, wwmax, nwaves, ncls, xi, xf,
                                          uout, umirror, b, sA);
}
template void launch_iface2d_wheels<double>(const LK&, const Tables&, const int32_t*, const int32_t*, const int32_t*,
                                            const int32_t*, const int32_t*, const double*, const int32_t*, int, int,
                                            const double*, const double*, double*, double*, const double*, double,
                                            hipStream_t);
template void launch_iface2d_wheels<float>(const LK&, const Tables&, const int32_t*, const int32_t*, const int32_t*,
                                           const int32_t*, const int32_t*, const double*, const int32_t*, int, int,
                                           const float*, const float*, float*, float*, const float*, double,
                                           hipStream_t);

// The same assembled residual rows from the interface tasks: one lane per (DoF, incident
// macro) pair forms its macro's term b_m - A_m x, the lanes of a DoF sum the terms in
// incidence order through shuffles, and the first lane (the lowest-id copy) stores the sum;
// the other copies, and every copy of a Dirichlet DoF, get 0.  Identical to k_iface_residual.
template <int D, typename Tin, typename Tout>
__global__ void __launch_bounds__(256) k_iface_residual_tasks(LK lk, Tables tb, const int32_t* __restrict__ tcopy,
                                                               const int32_t* __restrict__ tinfo,
                                                               const int32_t* __restrict__ tloc,
                                                               const int32_t* __restrict__ tseg,
                                                               const int32_t* __restrict__ wmax, int w0, int w1,
                                                               const Tin* __restrict__ x, const Tin* __restrict__ b,
                                                               Tout* __restrict__ y, double sA) {
  const int w = __builtin_amdgcn_readfirstlane(w0 + d_xcd_block() * 4 + (int)(threadIdx.x >> 6));
  if (w >= w1) return;
  const int lane = (int)(threadIdx.x & 63);
  const int idx = w * 64 + lane;
  const int cp = tcopy[idx];
  const int info = tinfo[idx], loc = tloc[idx], seg = tseg[idx];
  const bool live = cp >= 0;
  const bool dir = (info >> 28) & 1;
  Tin term = (Tin)0;
  if (live && !dir) {
    const int m = info & 0xffffff, mask = (info >> 24) & 15;
    const int i = loc & 2047, j = (loc >> 11) & 2047, k = loc >> 22;
    const int64_t base = (int64_t)m * lk.S;
    Tin o, dg;
    d_row_const<D, Tin>(lk, tb.stiff + ((size_t)m * kMaxMask + mask) * ndir<D>(), tb.validdirs[mask],
                        sA * tb.kappa[m], x, base, i, j, k, o, dg);
    term = b[cp] - o - dg * x[cp];
  }
  const int lead = seg & 63, len = seg >> 8;
  Tin r = (Tin)0;
  const int wm = wmax[w];
  for (int kq = 0; kq < wm; ++kq) {
    const Tin t = __shfl(term, min(lead + kq, 63), 64);
    if (kq < len) r += t;
  }
  if (live) y[cp] = (Tout)(lane == lead ? r : (Tin)0);
}

// Assembled residual rows at interface DoFs: r = sum_m (b_m - A_m x) in Tin precision, stored
// in the lowest-id copy (other copies 0, Dirichlet DoFs 0).  Used when a float64 residual is
// handed to float32 cycles: the per-macro partial rows are one-sided differences that cancel
// only after summation, so they are summed before rounding.
template <int D, typename Tin, typename Tout, bool P1>
__global__ void __launch_bounds__(256) k_iface_residual(LK lk, Tables tb, const Tin* __restrict__ x,
                                                         const Tin* __restrict__ b, Tout* __restrict__ y, double sA,
                                                         const double* __restrict__ kn) {
  const int64_t t = (int64_t)d_xcd_block() * 256 + threadIdx.x;
  if (t >= lk.nIface) return;
  int p, co[3], np;
  d_iface_decode(lk, tb, t, p, co, np);
  const int q0 = tb.inc_off[p], q1 = tb.inc_off[p + 1];
  const bool dir = tb.primdir[p] != 0;
  Tin r = (Tin)0;
  if (!dir) {
    for (int q = q0; q < q1; ++q) {
      const Inc in = tb.inc[q];
      int lc[4] = {0, 0, 0, 0};
      for (int rr = 0; rr < np; ++rr) lc[in.slot[rr]] = co[rr];
      const int64_t base = (int64_t)in.macro * lk.S;
      const int ctr = d_lin<D>(lk.n, lc[1], lc[2], lc[3]);
      Tin o, dg;
      if constexpr (P1) {
        d_row_p1<D, Tin>(lk, tb.elemK + (size_t)in.macro * ntype<D>() * (D + 1) * (D + 1), tb.incvalid[in.mask], sA,
                         kn, x, base, lc[1], lc[2], lc[3], o, dg);
      } else {
        d_row_const<D, Tin>(lk, tb.stiff + ((size_t)in.macro * kMaxMask + in.mask) * ndir<D>(),
                            tb.validdirs[in.mask], sA * tb.kappa[in.macro], x, base, lc[1], lc[2], lc[3], o, dg);
      }
      r += b[base + ctr] - o - dg * x[base + ctr];
    }
  }
  for (int q = q0; q < q1; ++q) {
    const Inc in = tb.inc[q];
    int lc[4] = {0, 0, 0, 0};
    for (int rr = 0; rr < np; ++rr) lc[in.slot[rr]] = co[rr];
    y[(int64_t)in.macro * lk.S + d_lin<D>(lk.n, lc[1], lc[2], lc[3])] = (Tout)(q == q0 ? r : (Tin)0);
  }
}

// ------------------------------------------------------------------------------------------
// value held by lane q+1 (from_next) or lane q-1 (from_prev) of the wavefront: full-wave DPP
// shifts (wave_shl:1 / wave_shr:1).  The end lanes get their own value back; callers discard
// them.
__device__ __forceinline__ float from_next(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_prev(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ double from_next(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false),
                          __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double from_prev(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false),
                          __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false));
}

// The cycle's prolongation fused into the first post-smoothing sweep of a 2D level: each loaded
// node gets u + (P e_c) (Dirichlet nodes keep u), exactly as the separate prolongation would
// store it, and every loaded node on the macro boundary is written to tout, where the interface
// classes of that sweep read their old values.  Every boundary node lies in the loaded region
// of some tile, and tiles that load the same node write the same value.
template <typename T>
struct ProLoad {
  __amdgpu_buffer_rsrc_t ec, tout;   // this macro's coarse correction (side nc) and boundary output
  int nc;
};

// boundary nodes of rows j0r .. j1r in the columns i0 .. i0 + 63: the store offset of node (i, j)
// if it is a macro-boundary node of the closure, else an offset past the buffer (the store is
// dropped); whether the region holds any boundary node at all is wave-uniform
__device__ __forceinline__ bool region_has_boundary(int n, int i0, int j0r, int j1r) {
  return i0 <= 0 || j0r <= 0 || i0 + 63 + j1r >= n;
}
template <typename T>
__device__ __forceinline__ uint32_t boundary_offset(int n, int i, int j) {
  // j is wave-uniform: row 0 is boundary in every column of the closure, rows 1 .. n only in
  // columns 0 and n - j
  const bool bnd = j == 0 ? (uint32_t)i <= (uint32_t)n : ((uint32_t)j <= (uint32_t)n && (i == 0 || i == n - j));
  return bnd ? (uint32_t)(d_lin2(n, 0, j) + i) * (uint32_t)sizeof(T) : 0xfffffff0u;
}

// rows jstart + r (r < NR, jstart of parity PAR) of lane column i, in u[]; only the rows
// R0 <= r < R1 hold loaded values.  Coarse row jc of the region is t = jc - (jstart >> 1).
// Every fine parity pattern takes its nodes from coarse columns i >> 1 (a) and (i + 1) >> 1
// (b; the same for even i).  Each lane loads its column a and takes b from the next lane; the
// last lane loads its b instead and takes its a from the lane before (for odd i), so every
// coarse value comes from one load per lane and row and DPP shifts.
template <typename T, int NR, int PAR, int R0, int R1>
__device__ __forceinline__ void pro_rows(int n, const ProLoad<T>& P, int i, int jstart, T* u) {
  constexpr int T0 = (R0 + PAR) >> 1, T1 = ((R1 - 1 + PAR) >> 1) + 2;   // coarse rows used
  const int q = (int)(threadIdx.x & 63);
  const int i0w = __builtin_amdgcn_readfirstlane(i - q);   // the wavefront's first column
  const bool iodd = (i & 1) != 0, last = q == 63;
  const int jcb = jstart >> 1, ic = last ? (i + 1) >> 1 : i >> 1, nc = P.nc;
  T A[T1];
#pragma unroll
  for (int t = T0; t < T1; ++t) {
    const int jc = jcb + t;
    const bool ok = ic >= 0 && jc >= 0 && ic + jc <= nc;
    d_bload(P.ec, ok ? (uint32_t)d_lin2(nc, ic, jc) * (uint32_t)sizeof(T) : 0xfffffff0u, A[t]);
  }
  // the coarse correction is zero on Dirichlet nodes (restriction clears it, no sweep writes
  // there), so P e adds exactly zero on fine Dirichlet nodes: no Dirichlet test is needed
  auto col_a = [&](int t) {
    const T pv = from_prev(A[t]);   // shifts run on every lane (a lane left out supplies nothing)
    return last && iodd ? pv : A[t];
  };
  auto col_b = [&](int t) {
    const T nx = from_next(A[t]);
    return iodd ? (last ? A[t] : nx) : A[t];
  };
#pragma unroll
  for (int r = R0; r < R1; ++r) {
    const int t = (r + PAR) >> 1;
    T lo, hi;
    if (((PAR + r) & 1) == 0) { lo = col_a(t); hi = col_b(t); }   // even row: along the row
    else { lo = col_b(t); hi = col_a(t + 1); }                       // odd row: along j, or the diagonal
    u[r] = u[r] + (T)0.5 * (lo + hi);
  }
  if (region_has_boundary(n, i0w, jstart + R0, jstart + R1 - 1)) {
#pragma unroll
    for (int r = R0; r < R1; ++r) d_bstore(P.tout, boundary_offset<T>(n, i, jstart + r), u[r]);
  }
}

// zero start (the first sweep of a cycle on a zero correction, without clearing it first): the
// loaded nodes are zeros, and the boundary nodes of rows R0 <= r < R1 are written as zeros to
// tout for the interface classes
template <typename T, int R0, int R1>
__device__ __forceinline__ void zero_rows(int n, const ProLoad<T>& P, int i, int jstart) {
  const int i0w = __builtin_amdgcn_readfirstlane(i - (int)(threadIdx.x & 63));
  if (!region_has_boundary(n, i0w, jstart + R0, jstart + R1 - 1)) return;
#pragma unroll
  for (int r = R0; r < R1; ++r) d_bstore(P.tout, boundary_offset<T>(n, i, jstart + r), (T)0);
}

// Fused Gauss-Seidel sweep over the macro-interior nodes of a 2D level: every interior colour
// class in one launch (the interface nodes stay fixed during this part of the sweep).  Each
// wavefront owns a core tile of (64 - 2C) columns x TS rows and loads it with a halo of C
// layers, one lane per column, every row of u and b into registers (all loads in flight at
// once, each row load contiguous).  Colour pass c updates the nodes of colour c at distance
// >= c+1 from the edge of the loaded region, reading row neighbours from the adjacent lanes
// through DPP shifts; those values equal what C class-by-class passes over the whole macro
// produce, because each pass only needs correct values one layer further out.  After C passes
// the core is exact and is written to uo; the halo work is redundant.  No LDS and no barriers.
template <typename T, int C, int TS, bool FINE, int MODE>
__device__ __forceinline__ void gs2d_wave_tile(int n, __amdgpu_buffer_rsrc_t um, __amdgpu_buffer_rsrc_t uom,
                                               __amdgpu_buffer_rsrc_t bm, int i0, int j0, int rb, int s1, int s2,
                                               T w1, T w2, T w3, T w4, T w5, T w6, T inv, const ProLoad<T>& P) {
  constexpr int H = C, RH = TS + 2 * H;
  const int q = threadIdx.x & 63;
  const int i = i0 + q;
  T ur[RH], br[RH];
  // branch-free loads: nodes outside the closure read the macro's first entry; no interior
  // update ever reads them.  um, bm, uom describe this macro's block (wave-uniform), the
  // per-lane offsets are 32-bit byte offsets.
  int roff = j0 * (n + 1) - (j0 * (j0 - 1)) / 2;
#pragma unroll
  for (int r = 0; r < RH; ++r) {
    const int j = j0 + r;
    const bool in = i >= 0 && j >= 0 && i + j <= n;
    // unsigned 32-bit byte offset from the wave-uniform base: scalar-base + vector-offset loads
    const uint32_t g = in ? (uint32_t)(roff + i) * (uint32_t)sizeof(T) : 0u;
    if constexpr (MODE == 2) ur[r] = (T)0;
    else d_bload(um, g, ur[r]);
    d_bload(bm, g, br[r]);
    roff += n + 1 - j;
  }
  if constexpr (MODE == 1) {
    if (j0 & 1) pro_rows<T, RH, 1, 0, RH>(n, P, i, j0, ur);
    else pro_rows<T, RH, 0, 0, RH>(n, P, i, j0, ur);
  } else if constexpr (MODE == 2) {
    zero_rows<T, 0, RH>(n, P, i, j0);
  }
  // colour of (i, j0): red-black parity or (i + 2 j) mod 3.  Row r has colour col0 + r s2
  // (mod 2) or col0 + 2 r (mod 3); with r and c compile-time constants the colour test is one
  // compare.  The update is a select, so every lane stays active for the DPP shifts.
  const int col0 = rb ? ((i * s1 + j0 * s2) & 1) : (((i + 2 * j0) % 3) + 3) % 3;
  // node (i, j0 + r) is interior iff rlo <= r <= rhi
  const int rhi = n - 1 - j0 - i, rlo = 1 - j0;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const bool lok = q >= c + 1 && q <= 62 - c && i >= 1;
    // re-materialise the per-lane bounds in each pass so the per-row compares are made where
    // they are used instead of being hoisted (and held) for every row at once
    int cl = col0, hi = rhi, lo = rlo;
    asm volatile("" : "+v"(cl), "+v"(hi), "+v"(lo));
    // neighbours from the adjacent lanes: from_next(row r) is the (i+1, j) value for row r and
    // the (i+1, j-1) value for row r+1; from_prev(row r+1) is the (i-1, j+1) value for row r and
    // the (i-1, j) value for row r+1.  Nodes of colour c never neighbour each other, so the
    // shifts taken before a row's update stay valid for the next row.
    T nx_dn = from_next(ur[c]);
    T pv_r = from_prev(ur[c + 1]);
#pragma unroll
    for (int r = c + 1; r <= RH - 2 - c; ++r) {
      const T nx_r = from_next(ur[r]);
      const T pv_up = from_prev(ur[r + 1]);
      const T acc = w1 * nx_r + w2 * ur[r + 1] + w3 * pv_up + w4 * pv_r + w5 * ur[r - 1] + w6 * nx_dn;
      const T v = (br[r] - acc) * inv;
      bool act;
      if (rb) act = ((cl ^ ((r & 1) & s2)) == c);
      else act = (cl == ((c - 2 * r) % 3 + 3) % 3);
      act = act && lok && (r >= lo) && (r <= hi);
      ur[r] = act ? v : ur[r];
      nx_dn = nx_r;
      pv_r = pv_up;
    }
  }
  if (q >= H && q < 64 - H && i >= 1) {
    int ro = (j0 + H) * (n + 1) - ((j0 + H) * (j0 + H - 1)) / 2;
#pragma unroll
    for (int r = H; r < H + TS; ++r) {
      const int j = j0 + r;
      if (j >= 1 && i + j <= n - 1)
        d_bstore(uom, (uint32_t)(ro + i) * (uint32_t)sizeof(T), ur[r]);
      ro += n + 1 - j;
    }
  }
}

// Multicolour (C = 3) form of the wavefront tile with every lane busy in every pass.  Node
// (i, j) has colour (i + 2 j) mod 3, so a fixed row holds each colour in every third column
// only.  Lane i instead keeps row j0 - 3 + (i mod 3) + s in slot s: the nodes of one colour
// then sit in the same slots of all lanes (j0 = 1 mod 3 for every tile), and pass c updates
// the slots s = 2c + 2 (mod 3) of every lane.  Row neighbours come from the adjacent lanes: a
// lane offers, by its own column mod 3, the slot that holds the asking lane's row (right,
// left, up-left, down-right neighbours), and DPP shifts deliver it.  The valid region
// shrinks by one node per pass exactly as in the row-aligned form.
template <typename T, int TS, bool FINE, int MODE>
__device__ __forceinline__ void gs2d_wave_tile_mc3(int n, __amdgpu_buffer_rsrc_t um, __amdgpu_buffer_rsrc_t uom,
                                                   __amdgpu_buffer_rsrc_t bm, int i0, int j0, T w1, T w2, T w3, T w4,
                                                   T w5, T w6, T inv, const ProLoad<T>& P) {
  constexpr int H = 3, RH = TS + 2 * H, K = 3, RS = RH + K + 1;
  const int q = threadIdx.x & 63;
  const int i = i0 + q;
  const int rho = ((i % 3) + 3) % 3;
  // load rows j0 - K + t (t = 0 .. RS+1) aligned across lanes, so every load is one contiguous
  // row segment, then rotate in registers: slot s takes aligned row s + (i mod 3)
  T us[RS + 2], bs[RS + 2];
  {
    int j = j0 - K;
    int roff = j * (n + 1) - (j * (j - 1)) / 2;
#pragma unroll
    for (int t = 0; t < RS + 2; ++t) {
      const int r = t - K;   // row of the loaded region, 0 .. RH-1
      const bool in = r >= 0 && r < RH && i >= 0 && j >= 0 && i + j <= n;
      const uint32_t g = in ? (uint32_t)(roff + i) * (uint32_t)sizeof(T) : 0u;
      if constexpr (MODE == 2) us[t] = (T)0;
      else d_bload(um, g, us[t]);
      d_bload(bm, g, bs[t]);
      roff += n + 1 - j;
      ++j;
    }
    // the aligned rows t = K .. K + RH - 1 are the loaded ones (the others hold placeholders)
    if constexpr (MODE == 1) {
      if ((j0 - K) & 1) pro_rows<T, RS + 2, 1, K, K + RH>(n, P, i, j0 - K, us);
      else pro_rows<T, RS + 2, 0, K, K + RH>(n, P, i, j0 - K, us);
    } else if constexpr (MODE == 2) {
      zero_rows<T, K, K + RH>(n, P, i, j0 - K);
    }
    const bool p1 = rho == 1, p2 = rho == 2;
#pragma unroll
    for (int t = 0; t < RS; ++t) {
      us[t] = p2 ? us[t + 2] : (p1 ? us[t + 1] : us[t]);
      bs[t] = p2 ? bs[t + 2] : (p1 ? bs[t + 1] : bs[t]);
    }
  }
  // node (i, j0 + r) is interior iff rlo <= r <= rhi
  const int rhi = n - 1 - j0 - i, rlo = 1 - j0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const bool lok = q >= c + 1 && q <= 62 - c && i >= 1;
    int rr = rho, hi = rhi, lo = rlo;
    asm volatile("" : "+v"(rr), "+v"(hi), "+v"(lo));
    const bool r0 = rr == 0, r2 = rr == 2;
#pragma unroll
    for (int s = 2; s <= RS - 3; ++s) {
      if (s % 3 != (2 * c + 2) % 3) continue;
      const int r = s - K + rr;
      const T sR = r0 ? us[s + 2] : us[s - 1];
      const T sL = r2 ? us[s - 2] : us[s + 1];
      const T sUL = r2 ? us[s - 1] : us[s + 2];
      const T sDR = r0 ? us[s + 1] : us[s - 2];
      const T acc = w1 * from_next(sR) + w2 * us[s + 1] + w3 * from_prev(sUL) + w4 * from_prev(sL) + w5 * us[s - 1] +
                    w6 * from_next(sDR);
      const T v = (bs[s] - acc) * inv;
      const bool act = lok && r >= c + 1 && r <= RH - 2 - c && r >= lo && r <= hi;
      us[s] = act ? v : us[s];
    }
  }
  if (q >= H && q < 64 - H && i >= 1) {
    // rotate back: aligned row r sits in slot r + K - (i mod 3)
    const bool p1 = rho == 1, p2 = rho == 2;
    int j = j0 + H;
    int roff = j * (n + 1) - (j * (j - 1)) / 2;
#pragma unroll
    for (int r = H; r < H + TS; ++r) {
      const T v = p2 ? us[r + K - 2] : (p1 ? us[r + K - 1] : us[r + K]);
      if (j >= 1 && i + j <= n - 1) d_bstore(uom, (uint32_t)(roff + i) * (uint32_t)sizeof(T), v);
      roff += n + 1 - j;
      ++j;
    }
  }
}

// one wavefront per tile of (64 - 2C) columns x TJ rows, processed as SUB consecutive
// sub-tiles of TJ/SUB rows.  Reads u, writes the interior of uo: tiles overlap in their
// halos, so an in-place update would let one tile read rows another tile has already
// written.  Blocks are spread over the XCDs in contiguous runs of tiles (block b runs on
// XCD b mod 8), so neighbouring tiles share their halo rows in one L2.
template <typename T, int C, int TJ, int SUB, bool FINE, int MODE>
__global__ void __launch_bounds__(256) k_gs2d_fused(LK lk, Tables tb, const T* __restrict__ u, T* __restrict__ uo,
                                                     const T* __restrict__ b,
                                                     const int32_t* __restrict__ tiles, int ntiles, int rb, double sA,
                                                     const T* __restrict__ ec, int cS, T* __restrict__ tout) {
  constexpr int H = C, TI = 64 - 2 * H, TS = TJ / SUB;
  const int per_xcd = (int)(gridDim.x >> 3);   // gridDim.x is a multiple of 8
  const int blk = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  // tile, macro and tile origin are uniform over the wavefront: keep them in scalar registers
  const int gt = __builtin_amdgcn_readfirstlane(blk * 4 + (int)(threadIdx.x >> 6));
  if (gt >= lk.nmacro * ntiles) return;
  const int m = gt / ntiles;
  const int tile = __builtin_amdgcn_readfirstlane(tiles[gt - m * ntiles]);
  const int64_t base = (int64_t)m * lk.S;
  const uint32_t bytes = (uint32_t)lk.Sraw * (uint32_t)sizeof(T);
  const int i0 = 1 + (tile & 0xffff) * TI - H;
  const double* W = tb.stiff + (size_t)m * kMaxMask * 7;
  const double ks = sA * tb.kappa[m];
  const T w1 = (T)(ks * W[1]), w2 = (T)(ks * W[2]), w3 = (T)(ks * W[3]);
  const T w4 = (T)(ks * W[4]), w5 = (T)(ks * W[5]), w6 = (T)(ks * W[6]);
  const T inv = (T)(1.0 / (ks * W[0]));
  const int s1 = rb ? tb.rbpar[m * 4 + 1] : 0, s2 = rb ? tb.rbpar[m * 4 + 2] : 0;
  ProLoad<T> P{};
  if constexpr (MODE == 1) {
    const int nc = lk.n >> 1;
    P.ec = d_rsrc(ec + (int64_t)m * cS, (uint32_t)(((nc + 1) * (nc + 2)) / 2) * (uint32_t)sizeof(T));
    P.nc = nc;
  }
  if constexpr (MODE != 0) P.tout = d_rsrc(tout + base, bytes);
#pragma unroll
  for (int sub = 0; sub < SUB; ++sub) {
    const int j0 = 1 + (tile >> 16) * TJ + sub * TS - H;
    if (j0 + H > lk.n - 2) break;
    if constexpr (C == 3 && TJ % 3 == 0 && TS % 3 == 0)
      gs2d_wave_tile_mc3<T, TS, FINE, MODE>(lk.n, d_rsrc(u + base, bytes), d_rsrc(uo + base, bytes),
                                           d_rsrc(b + base, bytes), i0, j0, w1, w2, w3, w4, w5, w6, inv, P);
    else
      gs2d_wave_tile<T, C, TS, FINE, MODE>(lk.n, d_rsrc(u + base, bytes), d_rsrc(uo + base, bytes),
                                          d_rsrc(b + base, bytes), i0, j0, rb, s1, s2, w1, w2, w3, w4, w5, w6, inv, P);
  }
}

// Fused Gauss-Seidel sweep over the interior of small 3D macros: one block per macro holds the
// whole closure of u in LDS and runs every interior colour pass there; b is read once per
// update from global memory.
template <typename T, int C, bool FINE>
__global__ void __launch_bounds__(1024) k_gs3d_macro(LK lk, Tables tb, T* __restrict__ u, const T* __restrict__ b,
                                                      const uint32_t* __restrict__ itab_all,
                                                      const int32_t* __restrict__ itab_off, int rb, double sA) {
  extern __shared__ unsigned char smem_raw[];
  T* su = reinterpret_cast<T*>(smem_raw);
  const int m = blockIdx.x;
  const int n = lk.n;
  const int64_t base = (int64_t)m * lk.S;
  for (int s = threadIdx.x; s < lk.Sraw; s += blockDim.x) su[s] = u[base + s];
  __syncthreads();
  const double* W = tb.stiff + (size_t)m * kMaxMask * 15;
  const double ks = sA * tb.kappa[m];
  T w[15];
#pragma unroll
  for (int q = 0; q < 15; ++q) w[q] = (T)(ks * W[q]);
  // the interior points of this macro's parity pattern, sorted by colour
  const int* rp = tb.rbpar + m * 4;
  const int pat = rb ? ((rp[1] & 1) | ((rp[2] & 1) << 1) | ((rp[3] & 1) << 2)) : 0;
  const uint32_t* itab = itab_all + (size_t)pat * lk.NI;
  const int32_t* off = itab_off + pat * (C + 1);
  for (int c = 0; c < C; ++c) {
    for (int t = off[c] + (int)threadIdx.x; t < off[c + 1]; t += blockDim.x) {
      const uint32_t pk = itab[t];
      const int i = pk & 1023, j = (pk >> 10) & 1023, k = pk >> 20;
      T acc = (T)0;
#pragma unroll
      for (int q = 1; q < 15; ++q) acc += w[q] * su[d_lin<3>(n, i + kOff3[q][0], j + kOff3[q][1], k + kOff3[q][2])];
      const int ctr = d_lin<3>(n, i, j, k);
      su[ctr] = (b[base + ctr] - acc) / w[0];
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < lk.NI; t += blockDim.x) {
    const uint32_t pk = itab[t];
    const int ctr = d_lin<3>(n, pk & 1023, (pk >> 10) & 1023, pk >> 20);
    u[base + ctr] = su[ctr];
  }
}

// ------------------------------------------------------------------------------------------
// y = alpha * b + beta * (A_m x) per macro over the closure (dual output); zero on Dirichlet
// nodes when zero_dir.  op 0: stiffness (scaled by kappa), 1: mass.
template <int D, typename Tin, typename Tout, bool P1>
__device__ __forceinline__ void apply_point(const LK& lk, const Tables& tb, const Tin* __restrict__ x,
                                            const Tin* __restrict__ b, Tout* __restrict__ y, int op, double scale,
                                            double alpha, double beta, int zero_dir, const double* __restrict__ kn, int m,
                                            int s) {
  int i, j, k;
  d_dec<D>(lk.n, s, i, j, k);
  const int mask = d_mask<D>(lk.n, i, j, k);
  const int64_t base = (int64_t)m * lk.S;
  if (zero_dir && ((tb.dirbits[m] >> mask) & 1)) { y[base + s] = (Tout)0; return; }
  Tin off, diag;
  if (op == 0) {
    if constexpr (P1) {
      d_row_p1<D, Tin>(lk, tb.elemK + (size_t)m * ntype<D>() * (D + 1) * (D + 1), tb.incvalid[mask], scale, kn, x, base,
                       i, j, k, off, diag);
    } else {
      d_row_const<D, Tin>(lk, tb.stiff + ((size_t)m * kMaxMask + mask) * ndir<D>(), tb.validdirs[mask],
                          scale * tb.kappa[m], x, base, i, j, k, off, diag);
    }
  } else {
    d_row_const<D, Tin>(lk, tb.mass + ((size_t)m * kMaxMask + mask) * ndir<D>(), tb.validdirs[mask], scale, x, base, i,
                        j, k, off, diag);
  }
  const Tin ax = off + diag * x[base + s];
  Tin v = (Tin)beta * ax;
  if (b) v += (Tin)alpha * b[base + s];
  y[base + s] = (Tout)v;
}

template <int D, typename Tin, typename Tout, bool P1>
__global__ void __launch_bounds__(256) k_apply(LK lk, Tables tb, const Tin* __restrict__ x, const Tin* __restrict__ b,
                                                Tout* __restrict__ y, int op, double scale, double alpha, double beta,
                                                int zero_dir, const double* __restrict__ kn) {
  const int nchunk = (lk.Sraw + 255) >> 8;
  const int blk = d_xcd_block();
  const int m = blk / nchunk;
  const int s = (blk - m * nchunk) * 256 + threadIdx.x;
  if (m >= lk.nmacro || s >= lk.Sraw) return;
  apply_point<D, Tin, Tout, P1>(lk, tb, x, b, y, op, scale, alpha, beta, zero_dir, kn, m, s);
}

// 3D y = alpha b + beta (A_m x) per macro by rows: one wavefront per closure row (j, k) of one
// macro, lanes along i in segments of 64.  Interior points take the macro's full stencil
// through wave-uniform neighbour-row offsets; points on the macro boundary take the partial
// stencil of their zero-set.  Same arithmetic, in the same order, as k_apply.
template <typename Tin, typename Tout>
__global__ void __launch_bounds__(256) k_apply3d_rows(LK lk, Tables tb, const Tin* __restrict__ x,
                                                       const Tin* __restrict__ b, Tout* __restrict__ y, int op,
                                                       double scale, double alpha, double beta, int zero_dir,
                                                       int nrows) {
  const int per_xcd = (int)(gridDim.x >> 3);   // gridDim.x is a multiple of 8
  const int blk = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  const int wid = __builtin_amdgcn_readfirstlane(blk * 4 + (int)(threadIdx.x >> 6));
  if (wid >= lk.nmacro * nrows) return;
  const int n = lk.n;
  const int m = wid / nrows;
  const int r = wid - m * nrows;
  // plane k holds the rows j = 0 .. n - k: r = sum_{k' < k} (n + 1 - k') + j
  const float a = 2.0f * (float)n + 3.0f;
  int k = (int)floorf(0.5f * (a - sqrtf(fmaxf(a * a - 8.0f * (float)r, 0.0f))));
  k = max(0, min(k, n));
  auto first = [&](int kk) { return kk * (n + 1) - (kk * (kk - 1)) / 2; };
  while (k < n && first(k + 1) <= r) ++k;
  while (k > 0 && first(k) > r) --k;
  const int j = r - first(k);
  const int64_t base = (int64_t)m * lk.S;
  auto row = [&](int jj, int kk) { return d_tet(n) - d_tet(n - kk) + jj * (n - kk + 1) - (jj * (jj - 1)) / 2; };
  const double* Wt = (op == 0 ? tb.stiff : tb.mass) + (size_t)m * kMaxMask * 15;
  const double sc = op == 0 ? scale * tb.kappa[m] : scale;
  Tin cq[15];
  int64_t ro[15];
  const bool inner_row = j >= 1 && k >= 1 && j + k <= n - 2;
#pragma unroll
  for (int q = 0; q < 15; ++q) {
    cq[q] = (Tin)(sc * Wt[q]);
    ro[q] = inner_row ? base + row(j + kOff3[q][1], k + kOff3[q][2]) + kOff3[q][0] : 0;
  }
  const int64_t r0 = base + row(j, k);
  const int len = n - j - k;   // points i = 0 .. len
  const uint32_t dirb = tb.dirbits[m];
  const int lane = (int)(threadIdx.x & 63);
  // chunks of 62 points: lane l owns i = 62 c + l - 1 (lanes 1 .. 62); the 14 neighbours of an
  // inner point lie in 7 rows, each loaded once per lane, the i +- 1 ones reached by full-wave
  // lane shifts (lanes 0 and 63 only load)
  const int nchunk = (len + 1 + 61) / 62;
  for (int c = 0; c < nchunk; ++c) {
    const int i = 62 * c + lane - 1;
    Tin v0 = (Tin)0, v2 = (Tin)0, v3 = (Tin)0, v6 = (Tin)0, v9 = (Tin)0, v10 = (Tin)0, v13 = (Tin)0;
    if (inner_row) {
      // row (j + dj, k + dk) holds i = 0 .. n - j - dj - k - dk
      auto ld = [&](int q, int dj, int dk) {
        const int ii = i - kOff3[q][0];
        return (ii >= 0 && ii <= n - j - dj - k - dk) ? x[ro[q] + i] : (Tin)0;
      };
      v0 = ld(0, 0, 0);
      v2 = ld(2, 1, 0);
      v3 = ld(3, 0, 1);
      v6 = ld(6, -1, 1);
      v9 = ld(9, -1, 0);
      v10 = ld(10, 0, -1);
      v13 = ld(13, 1, -1);
    }
    // neighbours by direction (kOff3 order): shifts run on every lane
    const Tin nb[15] = {v0, from_next(v0), v2, v3, from_prev(v2), from_prev(v3), v6, from_next(v6),
                        from_prev(v0), v9, v10, from_next(v9), from_next(v10), v13, from_prev(v13)};
    if (lane < 1 || lane > 62 || i > len) continue;
    const int mask = d_mask<3>(n, i, j, k);
    const int64_t ctr = r0 + i;
    if (zero_dir && ((dirb >> mask) & 1)) { y[ctr] = (Tout)0; continue; }
    Tin off, diag;
    if (mask == 0) {
      Tin acc = (Tin)0;
#pragma unroll
      for (int q = 1; q < 15; ++q) acc += cq[q] * nb[q];
      off = acc;
      diag = cq[0];
    } else {
      d_row_const<3, Tin>(lk, Wt + (size_t)mask * 15, tb.validdirs[mask], sc, x, base, i, j, k, off, diag);
    }
    const Tin ax = off + diag * x[ctr];
    Tin v = (Tin)beta * ax;
    if (b) v += (Tin)alpha * b[ctr];
    y[ctr] = (Tout)v;
  }
}

// 2D y = alpha b + beta (A_m x) with a per-macro coefficient in two wavefront roles of one
// launch.  Interior role (wavefronts 0 .. nint-1): a 62-node segment of kApplyRowsOp rows of one
// macro, lanes along i, the macro's full stencil with weights computed once per wavefront;
// each lane loads its column of the kApplyRowsOp + 2 rows once, all before the arithmetic, and
// takes the neighbours along i from the adjacent lanes; nodes on the macro boundary are left
// to the other role.  Boundary role: one lane per boundary node (3n per macro: row j = 0,
// column i = 0, the edge i + j = n) with its partial stencil.  x and y are accessed through
// buffer descriptors bounded to the macro block.
constexpr int kApplyRows = 4;    // rows per wavefront of the transfer kernels
constexpr int kApplyRowsOp = 8;  // rows per wavefront of the operator application
template <typename Tin, typename Tout>
__global__ void __launch_bounds__(256) k_apply2d_rows(LK lk, Tables tb, const Tin* __restrict__ x,
                                                      const Tin* __restrict__ b, Tout* __restrict__ y, int op,
                                                      double scale, double alpha, double beta, int zero_dir, int nseg,
                                                      int nint) {
  constexpr int R = kApplyRowsOp;
  const int n = lk.n;
  const int nrb = (n + 1 + R - 1) / R;
  const int wid = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + (int)(threadIdx.x >> 6));
  const int lane = (int)(threadIdx.x & 63);
  if (wid >= nint) {
    // boundary role
    const int64_t t = (int64_t)(wid - nint) * 64 + lane;
    if (t >= (int64_t)lk.nmacro * 3 * n) return;
    const int m = (int)(t / (3 * n));
    const int q = (int)(t - (int64_t)m * 3 * n);
    int i, j;
    if (q <= n) { i = q; j = 0; }
    else if (q <= 2 * n) { i = 0; j = q - n; }
    else { j = q - 2 * n; i = n - j; }
    const int mask = d_mask<2>(n, i, j, 0);
    const int64_t base = (int64_t)m * lk.S;
    const int s = d_lin2(n, i, j);
    if (zero_dir && ((tb.dirbits[m] >> mask) & 1)) { y[base + s] = (Tout)0; return; }
    Tin off, diag;
    const double* W = (op == 0 ? tb.stiff : tb.mass) + ((size_t)m * kMaxMask + mask) * 7;
    d_row_const<2, Tin>(lk, W, tb.validdirs[mask], op == 0 ? scale * tb.kappa[m] : scale, x, base, i, j, 0, off, diag);
    Tin v = (Tin)beta * (off + diag * x[base + s]);
    if (b) v += (Tin)alpha * b[base + s];
    y[base + s] = (Tout)v;
    return;
  }
  const int m = wid / (nrb * nseg);
  const int rem = wid - m * nrb * nseg;
  const int jb = rem / nseg, seg = rem - jb * nseg;
  if (seg * 62 > n - jb * R) return;   // the segment starts beyond the first row's end
  // lanes 1 .. 62 own the points i = seg * 62 + lane - 1; lanes 0 and 63 only load the
  // neighbours i - 1 and i + 1 of the end lanes, which reach them by full-wave lane shifts
  const int i = seg * 62 + lane - 1;
  const int64_t base = (int64_t)m * lk.S;
  const __amdgpu_buffer_rsrc_t rx = d_rsrc(x + base, (uint32_t)lk.Sraw * (uint32_t)sizeof(Tin));
  const __amdgpu_buffer_rsrc_t ry = d_rsrc(y + base, (uint32_t)lk.Sraw * (uint32_t)sizeof(Tout));
  const __amdgpu_buffer_rsrc_t rbb = d_rsrc(b ? b + base : x + base, b ? (uint32_t)lk.Sraw * (uint32_t)sizeof(Tin) : 0u);
  const double* Wt = (op == 0 ? tb.stiff : tb.mass) + (size_t)m * kMaxMask * 7;
  const double sc = op == 0 ? scale * tb.kappa[m] : scale;
  Tin w[7];
#pragma unroll
  for (int d = 0; d < 7; ++d) w[d] = (Tin)(sc * Wt[d]);
  // rows jb R - 1 .. jb R + R of x at column i (zero outside the closure)
  Tin xr[R + 2];
#pragma unroll
  for (int q = 0; q < R + 2; ++q) {
    const int j = jb * R - 1 + q;
    const bool in = j >= 0 && j <= n && i >= 0 && i <= n - j;
    Tin v;
    d_bload(rx, in ? (uint32_t)(d_lin2(n, 0, j) + i) * (uint32_t)sizeof(Tin) : 0u, v);
    xr[q] = in ? v : (Tin)0;
  }
  // b of the wavefront's own rows, loaded with x (past the closure, or without b through an
  // empty descriptor: zeros), so no row waits for a load of its own
  Tin br[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = jb * R + r;
    const bool in = j <= n && i >= 0 && i <= n - j;
    d_bload(rbb, in ? (uint32_t)(d_lin2(n, 0, j) + i) * (uint32_t)sizeof(Tin) : 0xfffffff0u, br[r]);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = jb * R + r;
    const Tin xc = xr[r + 1], xu = xr[r + 2], xd = xr[r];
    // neighbours in the order of the stencil directions (i+1,j) (i,j+1) (i-1,j+1) (i-1,j)
    // (i,j-1) (i+1,j-1); the shifts run on every lane
    const Tin nb[7] = {xc, from_next(xc), xu, from_prev(xu), from_prev(xc), xd, from_next(xd)};
    const bool ok = lane >= 1 && lane <= 62 && j >= 1 && i >= 1 && i + j <= n - 1;
    const int ctr = d_lin2(n, 0, j) + i;
    Tin off = (Tin)0;
#pragma unroll
    for (int d = 1; d < 7; ++d) off += w[d] * nb[d];
    Tin v = (Tin)beta * (off + w[0] * nb[0]);
    if (b) v += (Tin)alpha * br[r];
    // nodes not owned here take an offset past the buffer: the store is dropped
    d_bstore(ry, ok ? (uint32_t)ctr * (uint32_t)sizeof(Tout) : 0xfffffff0u, (Tout)v);
  }
}

// r_c = P^T r_f per macro (dual in, dual out); zero on coarse Dirichlet nodes.  Coarse closure
// point s of macro m (s < c.Sraw)
template <int D, typename T>
__device__ __forceinline__ void restrict_point(const LK& f, const LK& c, const Tables& tb, const T* __restrict__ rf,
                                               T* __restrict__ bc, int m, int s) {
  const int64_t cb = (int64_t)m * c.S, fb = (int64_t)m * f.S;
  int i, j, k;
  d_dec<D>(c.n, s, i, j, k);
  const int mask = d_mask<D>(c.n, i, j, k);
  if ((tb.dirbits[m] >> mask) & 1) { bc[cb + s] = (T)0; return; }
  const uint32_t valid = tb.validdirs[mask];
  const int fi = 2 * i, fj = 2 * j, fk = 2 * k;
  const NbrIdx<D> nb(f.n, fi, fj, fk);
  T acc = (T)0;
#pragma unroll
  for (int q = 1; q < ndir<D>(); ++q) {
    if (!((valid >> q) & 1)) continue;
    acc += rf[fb + nb.at(q)];
  }
  bc[cb + s] = rf[fb + d_lin<D>(f.n, fi, fj, fk)] + (T)0.5 * acc;
}

template <int D, typename T>
__global__ void __launch_bounds__(256) k_restrict(LK f, LK c, Tables tb, const T* __restrict__ rf, T* __restrict__ bc,
                                                   T* __restrict__ zc) {
  // grid over the padded coarse block; zc (if given) is cleared over the whole block: the
  // coarse correction of the next cycle starts from zero without a separate fill launch
  const int nchunk = (int)((c.S + 255) >> 8);
  const int blk = d_xcd_block();
  const int m = blk / nchunk;
  const int s = (blk - m * nchunk) * 256 + threadIdx.x;
  if (m >= c.nmacro) return;
  if (zc && s < c.S) zc[(int64_t)m * c.S + s] = (T)0;
  if (s >= c.Sraw) return;
  restrict_point<D, T>(f, c, tb, rf, bc, m, s);
}

// prolongation over the fine closure.  mode 0: uf += P ec on non-Dirichlet nodes;
// mode 1: uf = P ec everywhere; mode 2 (FMG): w = P ec, uf = P ec (g on Dirichlet nodes).
// Fine closure point s of macro m (s < f.Sraw)
template <int D, typename T>
__device__ __forceinline__ void prolong_point(const LK& f, const LK& c, const Tables& tb, const T* __restrict__ ec,
                                              T* __restrict__ uf, T* __restrict__ w, const T* __restrict__ g, int mode,
                                              int m, int s) {
  int i, j, k;
  d_dec<D>(f.n, s, i, j, k);
  const int64_t fb = (int64_t)m * f.S;
  const bool dir = (tb.dirbits[m] >> d_mask<D>(f.n, i, j, k)) & 1;
  if (mode == 0 && dir) return;
  const T v = d_prolong_val<D, T>(c.n, ec, (int64_t)m * c.S, i, j, k);
  if (mode == 0) uf[fb + s] += v;
  else if (mode == 1) uf[fb + s] = v;
  else {
    w[fb + s] = v;
    uf[fb + s] = dir ? g[fb + s] : v;
  }
}

template <int D, typename T>
__global__ void __launch_bounds__(256) k_prolong(LK f, LK c, Tables tb, const T* __restrict__ ec, T* __restrict__ uf,
                                                  T* __restrict__ w, const T* __restrict__ g, int mode) {
  const int nchunk = (f.Sraw + 255) >> 8;
  const int blk = d_xcd_block();
  const int m = blk / nchunk;
  const int s = (blk - m * nchunk) * 256 + threadIdx.x;
  if (m >= f.nmacro || s >= f.Sraw) return;
  prolong_point<D, T>(f, c, tb, ec, uf, w, g, mode, m, s);
}

// 2D prolongation by rows (modes as k_prolong): each wavefront takes a 64-node segment of
// kApplyRows consecutive fine rows of one macro; the coarse rows a fine row interpolates from
// are scalar, lanes differ only in their column.  Accesses go through descriptors bounded to
// the macro blocks.
template <typename T>
__global__ void __launch_bounds__(256) k_prolong2d_rows(LK f, LK c, Tables tb, const T* __restrict__ ec,
                                                        T* __restrict__ uf, T* __restrict__ w, const T* __restrict__ g,
                                                        int mode, int nseg) {
  constexpr int R = kApplyRows;
  const int n = f.n, nc = c.n;
  const int nrb = (n + 1 + R - 1) / R;
  const int wid = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + (int)(threadIdx.x >> 6));
  const int m = wid / (nrb * nseg);
  if (m >= f.nmacro) return;
  const int rem = wid - m * nrb * nseg;
  const int jb = rem / nseg, seg = rem - jb * nseg;
  if (seg * 64 > n - jb * R) return;
  const int i = seg * 64 + (int)(threadIdx.x & 63);
  const int64_t fb = (int64_t)m * f.S, cb = (int64_t)m * c.S;
  const __amdgpu_buffer_rsrc_t re = d_rsrc(ec + cb, (uint32_t)c.Sraw * (uint32_t)sizeof(T));
  const __amdgpu_buffer_rsrc_t ru = d_rsrc(uf + fb, (uint32_t)f.Sraw * (uint32_t)sizeof(T));
  const uint32_t dirb = tb.dirbits[m];
  T lo[R], hi[R], u0[R];
  int sidx[R];
  bool ok[R], dir[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = jb * R + r;
    ok[r] = j <= n && i < n + 1 - j;
    // the two coarse nodes of the lattice direction whose endpoints have this parity pattern
    // (one node, taken twice, when both fine indices are even)
    int ilo, jlo, ihi, jhi;
    if ((j & 1) == 0) {
      jlo = jhi = j >> 1;
      ilo = i >> 1;
      ihi = (i + 1) >> 1;
    } else if ((i & 1) == 0) {
      ilo = ihi = i >> 1;
      jlo = (j - 1) >> 1;
      jhi = (j + 1) >> 1;
    } else {
      ilo = (i + 1) >> 1;
      jlo = (j - 1) >> 1;
      ihi = (i - 1) >> 1;
      jhi = (j + 1) >> 1;
    }
    d_bload(re, ok[r] ? (uint32_t)d_lin2(nc, ilo, jlo) * (uint32_t)sizeof(T) : 0u, lo[r]);
    d_bload(re, ok[r] ? (uint32_t)d_lin2(nc, ihi, jhi) * (uint32_t)sizeof(T) : 0u, hi[r]);
    sidx[r] = ok[r] ? d_lin2(n, i, j) : 0;
    dir[r] = ok[r] && ((dirb >> d_mask<2>(n, i, j, 0)) & 1);
    if (mode == 0) d_bload(ru, (uint32_t)sidx[r] * (uint32_t)sizeof(T), u0[r]);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (!ok[r]) continue;
    const int j = jb * R + r;
    const T v = ((i | j) & 1) ? (T)0.5 * (lo[r] + hi[r]) : lo[r];
    const int s = sidx[r];
    const uint32_t fo = (uint32_t)s * (uint32_t)sizeof(T);
    if (mode == 0) {
      if (!dir[r]) d_bstore(ru, fo, u0[r] + v);
    } else if (mode == 1) {
      d_bstore(ru, fo, v);
    } else {
      w[fb + s] = v;
      d_bstore(ru, fo, dir[r] ? g[fb + s] : v);
    }
  }
}

// 2D restriction r_c = P^T r_f by rows of coarse nodes (as k_restrict, optional clearing of
// zc over the coarse block done by the same launch).  A wavefront takes kRestrictCols coarse
// columns of R = kRestrictRows coarse rows: lane l holds fine column 2 i0 - 1 + l of the 2R + 1
// fine rows around them (whole-row loads), and each odd lane, the centre 2i of one coarse node,
// takes the values of the fine columns 2i - 1 and 2i + 1 from the lanes beside it by DPP
// shifts.  Fine nodes outside the closure count as zero.  The seven terms are summed in the
// order of the lattice directions, as k_restrict does.
constexpr int kRestrictCols = 31, kRestrictRows = 8;
template <typename T>
__global__ void __launch_bounds__(256) k_restrict2d_rows(LK f, LK c, Tables tb, const T* __restrict__ rf,
                                                         T* __restrict__ bc, T* __restrict__ zc, int nseg) {
  constexpr int R = kRestrictRows, NF = 2 * R + 1;
  const int n = c.n, nf = f.n;
  const int nrb = (n + 1 + R - 1) / R;
  const int wid = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + (int)(threadIdx.x >> 6));
  const int m = wid / (nrb * nseg);
  if (m >= c.nmacro) return;
  const int rem = wid - m * nrb * nseg;
  const int jb = rem / nseg, seg = rem - jb * nseg;
  const int lane = (int)(threadIdx.x & 63);
  const int64_t fb = (int64_t)m * f.S, cb = (int64_t)m * c.S;
  // the padding of the coarse block (beyond the closure) is cleared by the wavefronts of the
  // first row block
  if (zc && jb == 0)
    for (int64_t s = c.Sraw + seg * 64 + lane; s < c.S; s += (int64_t)nseg * 64) zc[cb + s] = (T)0;
  const int j0 = jb * R, i0 = seg * kRestrictCols;
  if (i0 > n - j0) return;   // no coarse node of this wavefront lies in the closure
  const __amdgpu_buffer_rsrc_t rr = d_rsrc(rf + fb, (uint32_t)f.Sraw * (uint32_t)sizeof(T));
  const __amdgpu_buffer_rsrc_t rc = d_rsrc(bc + cb, (uint32_t)c.Sraw * (uint32_t)sizeof(T));
  const uint32_t dirb = tb.dirbits[m];
  // fine rows 2 j0 - 1 .. 2 (j0 + R - 1) + 1 at fine column a, every lane (the shifts need all)
  const int a = 2 * i0 - 1 + lane;
  T v[NF], vn[NF], vp[NF];
#pragma unroll
  for (int t = 0; t < NF; ++t) {
    const int b = 2 * j0 - 1 + t;
    const bool use = a >= 0 && b >= 0 && a + b <= nf;
    d_bload(rr, use ? (uint32_t)d_lin2(nf, a, b) * (uint32_t)sizeof(T) : 0u, v[t]);
    v[t] = use ? v[t] : (T)0;
  }
#pragma unroll
  for (int t = 0; t < NF; ++t) {
    vn[t] = from_next(v[t]);
    vp[t] = from_prev(v[t]);
  }
  const bool centre = (lane & 1) != 0 && lane < 2 * kRestrictCols;
  const int i = i0 + ((lane - 1) >> 1);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = j0 + r;
    if (!(centre && j <= n && i < n + 1 - j)) continue;
    const int s = d_lin2(n, i, j);
    const uint32_t co = (uint32_t)s * (uint32_t)sizeof(T);
    if (zc) zc[cb + s] = (T)0;
    if ((dirb >> d_mask<2>(n, i, j, 0)) & 1) {
      d_bstore(rc, co, (T)0);
      continue;
    }
    // rows 2j - 1, 2j, 2j + 1 are v[2r], v[2r + 1], v[2r + 2]; directions (1,0), (0,1),
    // (-1,1), (-1,0), (0,-1), (1,-1)
    T acc = (T)0;
    acc += vn[2 * r + 1];
    acc += v[2 * r + 2];
    acc += vp[2 * r + 2];
    acc += vp[2 * r + 1];
    acc += v[2 * r];
    acc += vn[2 * r];
    d_bstore(rc, co, v[2 * r + 1] + (T)0.5 * acc);
  }
}

// dst (level l) = src (level L) at the same points: nodal injection
template <int D>
__global__ void __launch_bounds__(256) k_inject(LK fine, LK coarse, const double* __restrict__ src, double* __restrict__ dst,
                                                 int shift) {
  const int nchunk = (coarse.Sraw + 255) >> 8;
  const int m = blockIdx.x / nchunk;
  const int s = (blockIdx.x - m * nchunk) * 256 + threadIdx.x;
  if (s >= coarse.Sraw) return;
  int i, j, k;
  d_dec<D>(coarse.n, s, i, j, k);
  dst[(int64_t)m * coarse.S + s] = src[(int64_t)m * fine.S + d_lin<D>(fine.n, i << shift, j << shift, k << shift)];
}

// x = g on Dirichlet nodes, `inner` elsewhere
template <int D>
__global__ void __launch_bounds__(256) k_init_dirichlet(LK lk, Tables tb, const double* __restrict__ g,
                                                         double* __restrict__ x, double inner) {
  const int nchunk = (lk.Sraw + 255) >> 8;
  const int m = blockIdx.x / nchunk;
  const int s = (blockIdx.x - m * nchunk) * 256 + threadIdx.x;
  if (s >= lk.Sraw) return;
  int i, j, k;
  d_dec<D>(lk.n, s, i, j, k);
  const int64_t base = (int64_t)m * lk.S;
  x[base + s] = ((tb.dirbits[m] >> d_mask<D>(lk.n, i, j, k)) & 1) ? g[base + s] : inner;
}

// x = g on Dirichlet nodes, unchanged elsewhere
template <int D>
__global__ void __launch_bounds__(256) k_impose_dirichlet(LK lk, Tables tb, const double* __restrict__ g,
                                                           double* __restrict__ x) {
  const int nchunk = (lk.Sraw + 255) >> 8;
  const int m = blockIdx.x / nchunk;
  const int s = (blockIdx.x - m * nchunk) * 256 + threadIdx.x;
  if (s >= lk.Sraw) return;
  int i, j, k;
  d_dec<D>(lk.n, s, i, j, k);
  const int64_t base = (int64_t)m * lk.S;
  if ((tb.dirbits[m] >> d_mask<D>(lk.n, i, j, k)) & 1) x[base + s] = g[base + s];
}

// 2D transfer of a level vector between two macro meshes of one domain: every closure node of
// the new mesh (coordinates as in k_dof_coords) is located in one of the candidate old macros
// of its macro (barycentric coordinates >= -1e-10), then in the old macro's lattice of side
// no, and gets the P1 interpolant of the old closure values on that micro triangle (NaN if no
// candidate contains it)
__global__ void __launch_bounds__(256) k_transfer2d(LK fn, const double* __restrict__ mxyz_new, LK fo,
                                                     const double* __restrict__ mxyz_old, const int32_t* __restrict__ coff,
                                                     const int32_t* __restrict__ cand, const double* __restrict__ uold,
                                                     double* __restrict__ unew) {
  const int nchunk = (fn.Sraw + 255) >> 8;
  const int m = blockIdx.x / nchunk;
  const int s = (blockIdx.x - m * nchunk) * 256 + threadIdx.x;
  if (s >= fn.Sraw) return;
  int i, j;
  d_dec2(fn.n, s, i, j);
  const double* X = mxyz_new + (size_t)m * 6;
  const double inv = 1.0 / fn.n;
  double x[2];
  for (int q = 0; q < 2; ++q) x[q] = X[q] + (i * inv) * (X[2 + q] - X[q]) + (j * inv) * (X[4 + q] - X[q]);
  double v = __builtin_nan("");
  for (int q = coff[m]; q < coff[m + 1]; ++q) {
    const int M = cand[q];
    const double* Y = mxyz_old + (size_t)M * 6;
    const double e1x = Y[2] - Y[0], e1y = Y[3] - Y[1], e2x = Y[4] - Y[0], e2y = Y[5] - Y[1];
    const double rx = x[0] - Y[0], ry = x[1] - Y[1];
    const double det = e1x * e2y - e1y * e2x;
    const double l1 = (rx * e2y - ry * e2x) / det, l2 = (e1x * ry - e1y * rx) / det;
    if (l1 < -1e-10 || l2 < -1e-10 || 1.0 - l1 - l2 < -1e-10) continue;
    const int no = fo.n;
    const double xi1 = l1 * no, xi2 = l2 * no;
    const int i0 = min(max((int)floor(xi1), 0), no - 1);
    const int j0 = min(max((int)floor(xi2), 0), no - 1 - i0);
    const double f1 = xi1 - i0, f2 = xi2 - j0;
    const double* U = uold + (int64_t)M * fo.S;
    if (f1 + f2 <= 1.0 || i0 + j0 + 2 > no)
      v = (1.0 - f1 - f2) * U[d_lin2(no, i0, j0)] + f1 * U[d_lin2(no, i0 + 1, j0)] + f2 * U[d_lin2(no, i0, j0 + 1)];
    else
      v = (f1 + f2 - 1.0) * U[d_lin2(no, i0 + 1, j0 + 1)] + (1.0 - f2) * U[d_lin2(no, i0 + 1, j0)] +
          (1.0 - f1) * U[d_lin2(no, i0, j0 + 1)];
    break;
  }
  unew[(int64_t)m * fn.S + s] = v;
}

// 3D transfer, one thread per closure node of the new level.  In a candidate old macro the
// point's barycentric coordinates (l1, l2, l3) (negative round-off clamped to zero) give lattice
// coordinates xi = no (l1, l2, l3); in cumulative form y = (xi1, xi1 + xi2, xi1 + xi2 + xi3),
// which is non-decreasing and at most no, the six micro-tetrahedron types of the lattice are
// the six Kuhn simplices of each unit cube base + [0,1]^3 (base = floor(y) clamped to 0..no-1).
// The point lies in the simplex that leaves base along the coordinates in order of decreasing
// fractional part f (ties: the later coordinate first, so every vertex stays non-decreasing and
// inside the closure), with P1 weights 1 - f_s0, f_s0 - f_s1, f_s1 - f_s2, f_s2.
__global__ void __launch_bounds__(256) k_transfer3d(LK fn, const double* __restrict__ mxyz_new, LK fo,
                                                     const double* __restrict__ mxyz_old, const int32_t* __restrict__ coff,
                                                     const int32_t* __restrict__ cand, const double* __restrict__ uold,
                                                     double* __restrict__ unew) {
  const int nchunk = (fn.Sraw + 255) >> 8;
  const int m = blockIdx.x / nchunk;
  const int s = (blockIdx.x - m * nchunk) * 256 + threadIdx.x;
  if (s >= fn.Sraw) return;
  int i, j, k;
  d_dec<3>(fn.n, s, i, j, k);
  const double* X = mxyz_new + (size_t)m * 12;
  const double inv = 1.0 / fn.n;
  double x[3];
  for (int q = 0; q < 3; ++q)
    x[q] = X[q] + (i * inv) * (X[3 + q] - X[q]) + (j * inv) * (X[6 + q] - X[q]) + (k * inv) * (X[9 + q] - X[q]);
  auto det3 = [](const double* a, const double* b, const double* c) {
    return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) + a[2] * (b[0] * c[1] - b[1] * c[0]);
  };
  double v = __builtin_nan("");
  for (int q = coff[m]; q < coff[m + 1]; ++q) {
    const int M = cand[q];
    const double* Y = mxyz_old + (size_t)M * 12;
    double e1[3], e2[3], e3[3], r[3];
    for (int a = 0; a < 3; ++a) {
      e1[a] = Y[3 + a] - Y[a];
      e2[a] = Y[6 + a] - Y[a];
      e3[a] = Y[9 + a] - Y[a];
      r[a] = x[a] - Y[a];
    }
    const double det = det3(e1, e2, e3);
    double l1 = det3(r, e2, e3) / det, l2 = det3(e1, r, e3) / det, l3 = det3(e1, e2, r) / det;
    if (l1 < -1e-10 || l2 < -1e-10 || l3 < -1e-10 || 1.0 - l1 - l2 - l3 < -1e-10) continue;
    l1 = fmax(l1, 0.0);
    l2 = fmax(l2, 0.0);
    l3 = fmax(l3, 0.0);
    const double ls = l1 + l2 + l3;
    if (ls > 1.0) {
      l1 /= ls;
      l2 /= ls;
      l3 /= ls;
    }
    const int no = fo.n;
    const double y[3] = {l1 * no, (l1 + l2) * no, fmin((l1 + l2 + l3) * no, (double)no)};
    int base[3], o[3] = {2, 1, 0};
    double f[3];
    for (int a = 0; a < 3; ++a) {
      base[a] = min(max((int)floor(y[a]), 0), no - 1);
      f[a] = y[a] - base[a];
    }
    // stable sort of (c, b, a) by decreasing fractional part
    for (int a = 1; a < 3; ++a)
      for (int b2 = a; b2 > 0 && f[o[b2]] > f[o[b2 - 1]]; --b2) {
        const int t = o[b2];
        o[b2] = o[b2 - 1];
        o[b2 - 1] = t;
      }
    const double w[4] = {1.0 - f[o[0]], f[o[0]] - f[o[1]], f[o[1]] - f[o[2]], f[o[2]]};
    const double* U = uold + (int64_t)M * fo.S;
    int cur[3] = {base[0], base[1], base[2]};
    double acc = 0.0;
    for (int t = 0; t < 4; ++t) {
      if (t > 0) ++cur[o[t - 1]];
      const int ii = min(max(cur[0], 0), no);
      const int jj = min(max(cur[1] - cur[0], 0), no - ii);
      const int kk = min(max(cur[2] - cur[1], 0), no - ii - jj);
      acc += w[t] * U[d_lin<3>(no, ii, jj, kk)];
    }
    v = acc;
    break;
  }
  unew[(int64_t)m * fn.S + s] = v;
}

// level 0: x (+)= A_II^{-1} (assembled rhs) on the inner coarse vertices; one thread per row
template <typename T>
__global__ void __launch_bounds__(256) k_coarse(int n0, const int32_t* __restrict__ coff, const int64_t* __restrict__ copy,
                                                 const double* __restrict__ Ainv, const T* __restrict__ rhs,
                                                 T* __restrict__ x, int accumulate) {
  extern __shared__ double sr[];
  for (int r = threadIdx.x; r < n0; r += blockDim.x) {
    double s = 0.0;
    for (int q = coff[r]; q < coff[r + 1]; ++q) s += (double)rhs[copy[q]];
    sr[r] = s;
  }
  __syncthreads();
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n0) return;
  double e = 0.0;
  for (int col = 0; col < n0; ++col) e += Ainv[(size_t)col * n0 + row] * sr[col];   // symmetric, coalesced
  for (int q = coff[row]; q < coff[row + 1]; ++q) {
    const int64_t ix = copy[q];
    x[ix] = accumulate ? (T)((double)x[ix] + e) : (T)e;
  }
}

// factored level-0 solve, x (+)= P^T X^T X P r with X = L^{-1} (column-major lower triangle,
// zeros above the diagonal) and perm[p] the inner vertex at position p.  Three launches:
// s = P r (summing each inner vertex's copies of the dual right-hand side), y = X s (one thread
// per row, columns in ascending order), x_p = (X^T y)_p (one workgroup per column p, a
// fixed-order block reduction) written to every copy of vertex perm[p]
template <typename T>
__global__ void __launch_bounds__(256) k_coarse_gather(int n0, const int32_t* __restrict__ coff,
                                                        const int64_t* __restrict__ copy,
                                                        const int32_t* __restrict__ perm, const T* __restrict__ rhs,
                                                        double* __restrict__ s) {
  const int p = (int)(blockIdx.x * 256 + threadIdx.x);
  if (p >= n0) return;
  const int r = perm[p];
  double t = 0.0;
  for (int q = coff[r]; q < coff[r + 1]; ++q) t += (double)rhs[copy[q]];
  s[p] = t;
}

__global__ void __launch_bounds__(256) k_coarse_fwd(int n0, const double* __restrict__ X, const double* __restrict__ s,
                                                     double* __restrict__ y) {
  const int i = (int)(blockIdx.x * 256 + threadIdx.x);
  // the wavefront's rows end at iw; X is zero above the diagonal, so the row sums need no
  // per-lane bounds inside the loop
  const int iw = min(n0 - 1, (int)(blockIdx.x * 256 + (threadIdx.x & ~63u)) + 63);
  const int ii = min(i, n0 - 1);
  double acc = 0.0;
  for (int j = 0; j <= iw; ++j) acc += X[(size_t)j * n0 + ii] * s[j];
  if (i < n0) y[i] = acc;
}

template <typename T>
__global__ void __launch_bounds__(256) k_coarse_bwd(int n0, const double* __restrict__ X, const double* __restrict__ y,
                                                     const int32_t* __restrict__ coff, const int64_t* __restrict__ copy,
                                                     const int32_t* __restrict__ perm, T* __restrict__ x,
                                                     int accumulate) {
  __shared__ double sh[4];
  const int p = (int)blockIdx.x;
  double acc = 0.0;
  for (int i = p + (int)threadIdx.x; i < n0; i += 256) acc += X[(size_t)p * n0 + i] * y[i];
  const double e = block_sum(acc, sh);
  if (threadIdx.x != 0) return;
  const int r = perm[p];
  for (int q = coff[r]; q < coff[r + 1]; ++q) {
    const int64_t ix = copy[q];
    x[ix] = accumulate ? (T)((double)x[ix] + e) : (T)e;
  }
}

// ------------------------------------------------------------------------------------------
// dense map of the cycle on one coarse level k: x_k = scatter(B gather(b_k)) with B row-major
// [rows][ld]; row and column r are inner DoF r of level k, gather sums a DoF's dual copies of
// b_k in their list order, scatter writes a row's value to every copy.
//
// Gather: one thread per DoF, all of its copy indices and then all of their values in flight
// at once (table entries past kmax, and the empty ones, read index 0 = none, whose value loads
// past the buffer and reads zero), summed in list order.
template <typename T, int KB>
__global__ void __launch_bounds__(256) k_dense_gather(int rows, int kmax, const int32_t* __restrict__ gat,
                                                       const T* __restrict__ b, int64_t nb, T* __restrict__ s) {
  const int r = (int)(blockIdx.x * 256 + threadIdx.x);
  if (r >= rows) return;
  const __amdgpu_buffer_rsrc_t rg = d_rsrc(gat, (uint32_t)((size_t)kmax * rows * 4));
  const __amdgpu_buffer_rsrc_t rb = d_rsrc(b, (uint32_t)((size_t)nb * sizeof(T)));
  int32_t id[KB];
#pragma unroll
  for (int q = 0; q < KB; ++q)
    id[q] = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rg, (uint32_t)(((size_t)q * rows + r) * 4), 0, 0);
  T v[KB];
#pragma unroll
  for (int q = 0; q < KB; ++q)
    d_bload(rb, id[q] > 0 ? (uint32_t)(id[q] - 1) * (uint32_t)sizeof(T) : 0xfffffff0u, v[q]);
  T acc = (T)0;
#pragma unroll
  for (int q = 0; q < KB; ++q) acc += v[q];
  s[r] = acc;
}

// Product: one wavefront per row, 16 rows per workgroup, the gathered b staged in LDS once per
// workgroup (zero past the rows).  A lane holds columns 256 q + 4 l .. + 3; the row is read in
// groups of dense_qc such chunks, each group's loads in flight at once (chunks past ld / 256 lie
// outside the row's buffer range and load zeros).  The row is summed in float64 in a fixed
// order, then written to every copy.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <typename T> constexpr int dense_qc() { return sizeof(T) == 4 ? 8 : 4; }

template <typename T>
__global__ void __launch_bounds__(1024) k_dense_map(int rows, int ld, const T* __restrict__ B,
                                                     const T* __restrict__ sg, const int32_t* __restrict__ off,
                                                     const int32_t* __restrict__ copy, T* __restrict__ x) {
  extern __shared__ unsigned char dense_smem[];
  T* sb = reinterpret_cast<T*>(dense_smem);
  constexpr int QC = dense_qc<T>(), W = (int)(4 * sizeof(T) / 16);   // 16-byte loads per 4 entries
  const int nq = ld / 256, nqr = (nq + QC - 1) / QC * QC;             // chunks, rounded to groups
  const int lane = (int)(threadIdx.x & 63), nw = (int)(blockDim.x >> 6);
  const int row = (int)blockIdx.x * nw + (int)(threadIdx.x >> 6);
  const int rr = __builtin_amdgcn_readfirstlane(min(row, rows - 1));   // uniform per wavefront
  const int o0 = off[rr], nc = off[rr + 1] - o0;
  const __amdgpu_buffer_rsrc_t rB = d_rsrc(B + (size_t)rr * ld, (uint32_t)((size_t)ld * sizeof(T)));
  // the gathered b into LDS: up to 8 loads per thread (rows <= 8192, blockDim = 1024)
  const __amdgpu_buffer_rsrc_t rs = d_rsrc(sg, (uint32_t)((size_t)rows * sizeof(T)));
  T g[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) d_bload(rs, (uint32_t)(((int)threadIdx.x + (int)blockDim.x * t) * (int)sizeof(T)), g[t]);
  const int32_t dst = lane < nc ? copy[o0 + lane] : -1;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int cc = (int)threadIdx.x + (int)blockDim.x * t;
    if (cc < nqr * 256) sb[cc] = g[t];
  }
  __syncthreads();
  double acc = 0.0;
  for (int q0 = 0; q0 < nq; q0 += QC) {
    u32x4 v[QC][W];
#pragma unroll
    for (int q = 0; q < QC; ++q)
#pragma unroll
      for (int h = 0; h < W; ++h)
        v[q][h] = __builtin_amdgcn_raw_buffer_load_b128(
            rB, (uint32_t)(((256 * (q0 + q) + 4 * lane) * (int)sizeof(T)) + 16 * h), 0, 0);
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      T e[4];
      __builtin_memcpy(e, &v[q][0], sizeof(e));
#pragma unroll
      for (int t = 0; t < 4; ++t) acc += (double)e[t] * (double)sb[256 * (q0 + q) + 4 * lane + t];
    }
  }
  // butterfly: at every step both partners add the same two values, so every lane ends with
  // bitwise the same sum and all copies get one value
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (row >= rows) return;
  if (dst >= 0) x[dst] = (T)acc;
  for (int q = o0 + 64 + lane; q < o0 + nc; q += 64) x[copy[q]] = (T)acc;
}

// one probe of the dense map: b = unit vector at level-vector index idx (n entries)
template <typename T>
__global__ void __launch_bounds__(256) k_unit(T* __restrict__ b, int64_t n, int64_t idx) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) b[i] = i == idx ? (T)1 : (T)0;
}

// the probe's result as column `probe` of the dense map: B[r][probe] = x at row r's first copy
template <typename T>
__global__ void __launch_bounds__(256) k_dense_harvest(int rows, const int32_t* __restrict__ off,
                                                        const int32_t* __restrict__ copy, int ld, int probe,
                                                        const T* __restrict__ x, T* __restrict__ B) {
  const int r = (int)(blockIdx.x * 256 + threadIdx.x);
  if (r >= rows) return;
  B[(size_t)r * ld + probe] = x[copy[off[r]]];
}

// ------------------------------------------------------------------------------------------
// reductions
// sum over macro-interior nodes of r^2 (per block partials)
template <int D>
__global__ void __launch_bounds__(256) k_sq_interior(LK lk, const double* __restrict__ r, double* __restrict__ partial) {
  // 2D: one wavefront per interior row (lanes along i); 3D (short rows): 256-entry chunks of
  // the contiguous macro blocks with a decode.  A fixed grid strides over all of them, one
  // partial per block: the sum order depends only on the sizes
  __shared__ double sh[4];
  const int n = lk.n;
  if constexpr (D == 3) {
    const int nch = (lk.Sraw + 255) >> 8;
    const int64_t nchunks = (int64_t)lk.nmacro * nch;
    double v3 = 0.0;
    for (int64_t g = blockIdx.x; g < nchunks; g += gridDim.x) {
      const int64_t m = g / nch;
      const int s = (int)(g - m * nch) * 256 + (int)threadIdx.x;
      if (s < lk.Sraw) {
        int i, j, k;
        d_dec<3>(n, s, i, j, k);
        if (d_mask<3>(n, i, j, k) == 0) {
          const double x = r[m * lk.S + s];
          v3 += x * x;
        }
      }
    }
    v3 = block_sum(v3, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = v3;
    return;
  }
  const int64_t rows = (int64_t)lk.nmacro * (n + 1) * (D == 3 ? (n + 1) : 1);
  const int64_t nw = (int64_t)gridDim.x * 4;
  const int lane = threadIdx.x & 63;
  double v = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); g < rows; g += nw) {
    int64_t m;
    int j, k = 0;
    if constexpr (D == 2) {
      m = g / (n + 1);
      j = (int)(g - m * (n + 1));
    } else {
      const int64_t jk = g % ((int64_t)(n + 1) * (n + 1));
      m = g / ((int64_t)(n + 1) * (n + 1));
      k = (int)(jk / (n + 1));
      j = (int)(jk - (int64_t)k * (n + 1));
      if (k < 1) continue;
    }
    const int ilast = n - 1 - j - k;   // interior nodes i = 1 .. ilast
    if (j < 1 || ilast < 1) continue;
    const int64_t rb = m * lk.S + d_lin<D>(n, 0, j, k);
    for (int i = 1 + lane; i <= ilast; i += 64) {
      const double x = r[rb + i];
      v += x * x;
    }
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = v;
}

// sum of squares over every closure entry (a vector whose interface rows are already
// assembled in one copy, all other copies and Dirichlet rows 0), accumulated in float64.  The
// closure of a macro is contiguous, so blocks stride over 256-entry chunks of the macro blocks
// (fixed grid, one partial per block).
template <int D, typename T>
__global__ void __launch_bounds__(256) k_sq_closure(LK lk, const T* __restrict__ r, double* __restrict__ partial) {
  __shared__ double sh[4];
  const int nch = (lk.Sraw + 255) >> 8;
  const int64_t nchunks = (int64_t)lk.nmacro * nch;
  double v = 0.0;
  for (int64_t g = blockIdx.x; g < nchunks; g += gridDim.x) {
    const int64_t m = g / nch;
    const int s = (int)(g - m * nch) * 256 + (int)threadIdx.x;
    if (s < lk.Sraw) {
      const double x = (double)r[m * lk.S + s];
      v += x * x;
    }
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = v;
}

// sum over non-Dirichlet interface DoFs of (sum of copies)^2 (dual vector)
template <int D>
__global__ void __launch_bounds__(256) k_sq_iface(LK lk, Tables tb, const double* __restrict__ r, double* __restrict__ partial) {
  __shared__ double sh[4];
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v = 0.0;
  if (t < lk.nIface) {
    int p, co[3], np;
    d_iface_decode(lk, tb, t, p, co, np);
    if (!tb.primdir[p]) {
      double s = 0.0;
      for (int q = tb.inc_off[p]; q < tb.inc_off[p + 1]; ++q) {
        const Inc in = tb.inc[q];
        int lc[4] = {0, 0, 0, 0};
        for (int rr = 0; rr < np; ++rr) lc[in.slot[rr]] = co[rr];
        s += r[(int64_t)in.macro * lk.S + d_lin<D>(lk.n, lc[1], lc[2], lc[3])];
      }
      v = s * s;
    }
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = v;
}

__global__ void __launch_bounds__(256) k_sum(const double* __restrict__ partial, int n, double* __restrict__ out) {
  __shared__ double sh[4];
  double v = 0.0;
  for (int q = threadIdx.x; q < n; q += 256) v += partial[q];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) *out = v;
}

// 2D L2 estimator by rows: per macro T the two sums of k_estimate<2, 0> (e1 = u - a on level
// L, e2 = u - P bc with bc on level L-1, each against T's mass matrix).  Interior role: one
// wavefront per block of kEstRows interior rows and 62 columns of one macro; every lane forms
// e1 and e2 at its column on the block's rows and the rows above and below (P bc evaluated once
// per node), and takes the values of columns i - 1 and i + 1 from its neighbour lanes.
// Boundary role: one lane per macro-boundary node with its partial mass stencil.  Every
// wavefront writes the two sums of its nodes to partial[(m * per-macro wavefronts + w) * 2 + v].
__global__ void __launch_bounds__(256) k_estimate2d_rows(LK f, LK c, Tables tb, const double* __restrict__ u,
                                                          const double* __restrict__ a,
                                                          const double* __restrict__ bc,
                                                          double* __restrict__ partial, double sM, int nrb, int nseg,
                                                          int nbw) {
  constexpr int R = kEstRows;
  const int wpm = nrb * nseg + nbw;
  const int wid = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + (int)(threadIdx.x >> 6));
  if (wid >= f.nmacro * wpm) return;
  const int m = wid / wpm;
  const int w = wid - m * wpm;
  const int n = f.n;
  const int lane = (int)(threadIdx.x & 63);
  const int64_t fb = (int64_t)m * f.S, cb = (int64_t)m * c.S;
  double s1 = 0.0, s2 = 0.0;
  if (w < nrb * nseg) {
    const int jb = w / nseg, seg = w - jb * nseg;
    const int j0 = 1 + jb * R;
    const int i = seg * 62 + lane;   // lanes 1 .. 62 produce; lanes 0 and 63 are halo
    const double* W = tb.mass + (size_t)m * kMaxMask * 7;
    double w7[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) w7[q] = W[q];
    double e1[R + 2], e2[R + 2];
#pragma unroll
    for (int t = 0; t < R + 2; ++t) {
      const int r = j0 - 1 + t;
      const bool in = r <= n && i <= n - r;
      double v1 = 0.0, v2 = 0.0;
      if (in) {
        const int q = d_lin2(n, i, r);
        const double uq = u[fb + q];
        v1 = uq - a[fb + q];
        v2 = uq - d_prolong_val<2, double>(c.n, bc, cb, i, r, 0);
      }
      e1[t] = v1;
      e2[t] = v2;
    }
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const int j = j0 + rr;
      // neighbours in the order of the 2D directions: (1,0) (0,1) (-1,1) (-1,0) (0,-1) (1,-1)
      const double a1 = w7[0] * e1[rr + 1] + w7[1] * from_next(e1[rr + 1]) + w7[2] * e1[rr + 2] +
                        w7[3] * from_prev(e1[rr + 2]) + w7[4] * from_prev(e1[rr + 1]) + w7[5] * e1[rr] +
                        w7[6] * from_next(e1[rr]);
      const double a2 = w7[0] * e2[rr + 1] + w7[1] * from_next(e2[rr + 1]) + w7[2] * e2[rr + 2] +
                        w7[3] * from_prev(e2[rr + 2]) + w7[4] * from_prev(e2[rr + 1]) + w7[5] * e2[rr] +
                        w7[6] * from_next(e2[rr]);
      if (lane >= 1 && lane <= 62 && i >= 1 && j <= n - 2 && i + j <= n - 1) {
        s1 += e1[rr + 1] * a1;
        s2 += e2[rr + 1] * a2;
      }
    }
  } else {
    const int q = (w - nrb * nseg) * 64 + lane;
    if (q < 3 * n) {
      int i, j;
      if (q <= n) { i = q; j = 0; }
      else if (q <= 2 * n) { i = 0; j = q - n; }
      else { j = q - 2 * n; i = n - j; }
      const int mask = d_mask<2>(n, i, j, 0);
      const double* W = tb.mass + ((size_t)m * kMaxMask + mask) * 7;
      const uint32_t valid = tb.validdirs[mask];
      double m1 = 0.0, m2 = 0.0;
      for (int d = 0; d < 7; ++d) {
        if (d && !((valid >> d) & 1)) continue;
        const int ii = i + kOff2[d][0], jj = j + kOff2[d][1];
        const int lq = d_lin2(n, ii, jj);
        const double uq = u[fb + lq];
        m1 += W[d] * (uq - a[fb + lq]);
        m2 += W[d] * (uq - d_prolong_val<2, double>(c.n, bc, cb, ii, jj, 0));
      }
      const int s = d_lin2(n, i, j);
      const double uc = u[fb + s];
      s1 = (uc - a[fb + s]) * m1;
      s2 = (uc - d_prolong_val<2, double>(c.n, bc, cb, i, j, 0)) * m2;
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    s1 += __shfl_xor(s1, o, 64);
    s2 += __shfl_xor(s2, o, 64);
  }
  if (lane == 0) {
    partial[((size_t)m * wpm + w) * 2 + 0] = s1 * sM;
    partial[((size_t)m * wpm + w) * 2 + 1] = s2 * sM;
  }
}

// Estimator: per macro T, sum over the closure nodes q of T of e(q) (N_T e)(q) for
// e1 = u - a (a on level L) and e2 = u - P bc (bc on level L-1), N_T the matrix of T's own
// micro elements for the chosen norm: NORM 0 the consistent mass matrix (L2), NORM 1 the
// stiffness matrix with the macro's coefficient (energy), NORM 2 the row-sum lumped mass
// matrix.  Per-block partials [macro][chunk][2].
template <int D, int NORM>
__global__ void __launch_bounds__(256) k_estimate(LK f, LK c, Tables tb, const double* __restrict__ u,
                                                   const double* __restrict__ a, const double* __restrict__ bc,
                                                   double* __restrict__ partial, double scale) {
  __shared__ double sh[4];
  const int nchunk = (f.Sraw + 255) >> 8;
  const int m = blockIdx.x / nchunk;
  const int chunk = blockIdx.x - m * nchunk;
  const int s = chunk * 256 + threadIdx.x;
  double v1 = 0.0, v2 = 0.0;
  if (s < f.Sraw) {
    int i, j, k;
    d_dec<D>(f.n, s, i, j, k);
    const int mask = d_mask<D>(f.n, i, j, k);
    const int64_t fb = (int64_t)m * f.S, cb = (int64_t)m * c.S;
    const double* W = (NORM == 1 ? tb.stiff : tb.mass) + ((size_t)m * kMaxMask + mask) * ndir<D>();
    const uint32_t valid = tb.validdirs[mask];
    const double sc = NORM == 1 ? scale * tb.kappa[m] : scale;
    const double uc = u[fb + s];
    const double e1c = uc - a[fb + s];
    const double e2c = uc - d_prolong_val<D, double>(c.n, bc, cb, i, j, k);
    double m1 = 0.0, m2 = 0.0;
    if constexpr (NORM == 2) {
      double rs = 0.0;
#pragma unroll
      for (int q = 0; q < ndir<D>(); ++q)
        if (!q || ((valid >> q) & 1)) rs += W[q];
      m1 = rs * e1c;
      m2 = rs * e2c;
    } else {
#pragma unroll
      for (int q = 0; q < ndir<D>(); ++q) {
        if (q && !((valid >> q) & 1)) continue;
        int o0, o1, o2;
        d_off<D>(q, o0, o1, o2);
        const int ii = i + o0, jj = j + o1, kk = k + o2;
        const int lq = d_lin<D>(f.n, ii, jj, kk);
        const double uq = u[fb + lq];
        const double e1 = uq - a[fb + lq];
        const double e2 = uq - d_prolong_val<D, double>(c.n, bc, cb, ii, jj, kk);
        m1 += W[q] * e1;
        m2 += W[q] * e2;
      }
    }
    v1 = e1c * m1 * sc;
    v2 = e2c * m2 * sc;
  }
  v1 = block_sum(v1, sh);
  v2 = block_sum(v2, sh);
  if (threadIdx.x == 0) {
    partial[((size_t)m * nchunk + chunk) * 2 + 0] = v1;
    partial[((size_t)m * nchunk + chunk) * 2 + 1] = v2;
  }
}

// per macro: sum over closure nodes of x(q) (A_m^unit y)(q) (unit-coefficient stiffness)
template <int D>
__global__ void __launch_bounds__(256) k_bilinear(LK lk, Tables tb, const double* __restrict__ x,
                                                   const double* __restrict__ y, double* __restrict__ partial, double sA) {
  __shared__ double sh[4];
  const int nchunk = (lk.Sraw + 255) >> 8;
  const int m = blockIdx.x / nchunk;
  const int chunk = blockIdx.x - m * nchunk;
  const int s = chunk * 256 + threadIdx.x;
  double v = 0.0;
  if (s < lk.Sraw) {
    int i, j, k;
    d_dec<D>(lk.n, s, i, j, k);
    const int mask = d_mask<D>(lk.n, i, j, k);
    const int64_t base = (int64_t)m * lk.S;
    double off, diag;
    d_row_const<D, double>(lk, tb.stiff + ((size_t)m * kMaxMask + mask) * ndir<D>(), tb.validdirs[mask], sA, y, base, i,
                           j, k, off, diag);
    v = x[base + s] * (off + diag * y[base + s]);
  }
  v = block_sum(v, sh);
  if (threadIdx.x == 0) partial[(size_t)m * nchunk + chunk] = v;
}

// out[m * nval + v] = sum over chunks (fixed order)
// one block per output (macro m, value v): the chunk partials of the macro summed by the block
__global__ void __launch_bounds__(256) k_macro_sum(const double* __restrict__ partial, int nmacro, int nchunk, int nval,
                                                   double* __restrict__ out) {
  __shared__ double sh[4];
  const int id = blockIdx.x;
  const int m = id / nval, v = id - m * nval;
  double s = 0.0;
  for (int q = (int)threadIdx.x; q < nchunk; q += 256) s += partial[((size_t)m * nchunk + q) * nval + v];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[id] = s;
}

// ------------------------------------------------------------------------------------------
// canonical <-> per-macro layout
// mode 0: primal (every copy gets the value); 1: dual (owner copy gets it, others 0);
// 2: dual with Dirichlet nodes zeroed
template <int D>
__global__ void __launch_bounds__(256) k_canon_to_full(LK lk, Tables tb, const double* __restrict__ canon,
                                                        double* __restrict__ full, int mode) {
  const int nchunk = (lk.Sraw + 255) >> 8;
  const int m = blockIdx.x / nchunk;
  const int s = (blockIdx.x - m * nchunk) * 256 + threadIdx.x;
  if (s >= lk.Sraw) return;
  int i, j, k;
  d_dec<D>(lk.n, s, i, j, k);
  const int mask = d_mask<D>(lk.n, i, j, k);
  double v = canon[d_canon<D>(lk, tb, m, i, j, k)];
  if (mode >= 1 && mask != 0 && !((tb.ownbits[m] >> mask) & 1)) v = 0.0;
  if (mode == 2 && ((tb.dirbits[m] >> mask) & 1)) v = 0.0;
  full[(int64_t)m * lk.S + s] = v;
}

// mode 0: primal (lowest-id copy); 1: dual (sum of copies)
template <int D>
__global__ void __launch_bounds__(256) k_full_to_canon(LK lk, Tables tb, const double* __restrict__ full,
                                                        double* __restrict__ canon, int mode) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= lk.ndof) return;
  if (t >= lk.nIface) {
    const int64_t u = t - lk.nIface;
    const int m = (int)(u / lk.NI);
    int i, j, k;
    d_dec<D>(lk.n - D - 1, (int)(u - (int64_t)m * lk.NI), i, j, k);
    canon[t] = full[(int64_t)m * lk.S + d_lin<D>(lk.n, i + 1, j + 1, k + (D == 3 ? 1 : 0))];
    return;
  }
  int p, co[3], np;
  d_iface_decode(lk, tb, t, p, co, np);
  double s = 0.0;
  const int q1 = mode == 0 ? tb.inc_off[p] + 1 : tb.inc_off[p + 1];
  for (int q = tb.inc_off[p]; q < q1; ++q) {
    const Inc in = tb.inc[q];
    int lc[4] = {0, 0, 0, 0};
    for (int r = 0; r < np; ++r) lc[in.slot[r]] = co[r];
    s += full[(int64_t)in.macro * lk.S + d_lin<D>(lk.n, lc[1], lc[2], lc[3])];
  }
  canon[t] = s;
}

// coordinates of canonical DoFs: x = x0 + sum_q (c_q / n)(x_q - x0) in the first adjacent macro
template <int D>
__global__ void __launch_bounds__(256) k_dof_coords(LK lk, Tables tb, const double* __restrict__ mxyz,
                                                     const int32_t* __restrict__ cells, double* __restrict__ xyz) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= lk.ndof) return;
  int m, lc[4] = {0, 0, 0, 0};
  if (t >= lk.nIface) {
    const int64_t u = t - lk.nIface;
    m = (int)(u / lk.NI);
    int i, j, k;
    d_dec<D>(lk.n - D - 1, (int)(u - (int64_t)m * lk.NI), i, j, k);
    lc[1] = i + 1; lc[2] = j + 1; lc[3] = D == 3 ? k + 1 : 0;
  } else {
    int p, co[3], np;
    d_iface_decode(lk, tb, t, p, co, np);
    const Inc in = tb.inc[tb.inc_off[p]];
    m = in.macro;
    for (int r = 0; r < np; ++r) lc[in.slot[r]] = co[r];
  }
  const double* X = mxyz + (size_t)m * (D + 1) * D;
  const double inv = 1.0 / lk.n;
  for (int q = 0; q < D; ++q) {
    double v = X[q];
    for (int a = 1; a <= D; ++a) v += (lc[a] * inv) * (X[a * D + q] - X[q]);
    xyz[t * D + q] = v;
  }
}

// ------------------------------------------------------------------------------------------
// elementwise
template <typename T>
__global__ void __launch_bounds__(256) k_fill(T* __restrict__ x, int64_t n, T v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] = v;
}
__global__ void __launch_bounds__(256) k_add_f32(double* __restrict__ u, const float* __restrict__ e, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) u[i] += (double)e[i];
}
__global__ void __launch_bounds__(256) k_copy(double* __restrict__ dst, const double* __restrict__ src, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// ------------------------------------------------------------------------------------------
// launchers
static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }
// grid of kernels that map blocks with d_xcd_block: padded to a multiple of 8
static inline unsigned grid8(int64_t blocks) { return (unsigned)((blocks + 7) / 8 * 8); }

#define HHG_DISPATCH_D(dim, F, ...) \
  do {                              \
    if ((dim) == 3) F<3> __VA_ARGS__; \
    else F<2> __VA_ARGS__;           \
  } while (0)

template <typename T>
void launch_smooth_interior(int dim, bool p1, const LK& lk, const Tables& tb, const T* uin, T* uout, const T* b, int colour,
                            int rb, int jacobi, double omega, double sA, const double* kn, bool fine, hipStream_t st) {
  if (lk.NI <= 0) return;
  if (dim == 3 && !p1 && !jacobi && uin == uout && lk.n >= max(lk.rows3d_min, 4)) {
    // Gauss-Seidel in place with a per-macro coefficient: by rows
    const int nrows = (lk.n - 3) * (lk.n - 2) / 2;
    const int64_t waves = (int64_t)lk.nmacro * nrows;
    const unsigned g = (unsigned)((waves + 31) / 32 * 8);   // 4 rows per block, a multiple of 8 blocks
    if (fine) k_gs3d_rows<T, true><<<g, 256, 0, st>>>(lk, tb, uout, b, colour, rb, sA, nrows);
    else k_gs3d_rows<T, false><<<g, 256, 0, st>>>(lk, tb, uout, b, colour, rb, sA, nrows);
    return;
  }
  const unsigned g = grid8((int64_t)lk.nmacro * ((lk.NI + 255) / 256));
#define HHG_SI(D, P, F) k_smooth_interior<D, T, P, F><<<g, 256, 0, st>>>(lk, tb, uin, uout, b, colour, rb, jacobi, omega, sA, kn)
  if (dim == 3) {
    if (p1) { if (fine) HHG_SI(3, true, true); else HHG_SI(3, true, false); }
    else { if (fine) HHG_SI(3, false, true); else HHG_SI(3, false, false); }
  } else {
    if (p1) { if (fine) HHG_SI(2, true, true); else HHG_SI(2, true, false); }
    else { if (fine) HHG_SI(2, false, true); else HHG_SI(2, false, false); }
  }
#undef HHG_SI
}

template <typename T>
bool launch_gs_fused(int dim, bool p1, const LK& lk, const Tables& tb, T* u, T* uo, const T* b, const int32_t* tiles,
                     int ntiles, const uint32_t* itab, const int32_t* itab_off, int rb, double sA, bool fine,
                     hipStream_t st, const T* pro_ec, int pro_cS, T* pro_t, bool zero_start) {
  if (p1 || lk.NI <= 0) return false;
  if (dim == 2) {
    if (ntiles <= 0) return false;
    const unsigned g = (unsigned)(((int64_t)lk.nmacro * ntiles + 31) / 32 * 8);   // 4 tiles per block, 8 XCDs
    const int mode = pro_ec ? 1 : (zero_start ? 2 : 0);
#define HHG_F2(C, N, F)                                                                                          \
  do {                                                                                                           \
    constexpr int TR = tile_rows(C, N);                                                                          \
    if (mode == 1)                                                                                               \
      k_gs2d_fused<T, C, TR, 1, F, 1><<<g, 256, 0, st>>>(lk, tb, u, uo, b, tiles, ntiles, rb, sA, pro_ec, pro_cS,     \
                                                         pro_t);                                                 \
    else if (mode == 2)                                                                                          \
      k_gs2d_fused<T, C, TR, 1, F, 2><<<g, 256, 0, st>>>(lk, tb, u, uo, b, tiles, ntiles, rb, sA, nullptr, 0, pro_t);  \
    else                                                                                                         \
      k_gs2d_fused<T, C, TR, 1, F, 0><<<g, 256, 0, st>>>(lk, tb, u, uo, b, tiles, ntiles, rb, sA, nullptr, 0,        \
                                                         nullptr);                                               \
  } while (0)
    // the kernel's tile height is the one the host built the tile table with
#define HHG_F2N(C, F)                                                               \
  do {                                                                              \
    if (tile_rows(C, lk.n) == tile_rows(C, kShortTileMaxN)) HHG_F2(C, kShortTileMaxN, F); \
    else HHG_F2(C, 2 * kShortTileMaxN, F);                                          \
  } while (0)
    if (rb) { if (fine) HHG_F2N(2, true); else HHG_F2N(2, false); }
    else { if (fine) HHG_F2N(3, true); else HHG_F2N(3, false); }
#undef HHG_F2N
#undef HHG_F2
    return true;
  }
  if (ntiles > 0 && lk.planes3d) {
    // red-black with per-macro coefficient, 16 <= n <= 64: whole planes in LDS, chunks of planes
    if (!rb || lk.n > kPlane3dMaxN) return false;
    const unsigned g = (unsigned)(((int64_t)lk.nmacro * ntiles + 7) / 8 * 8);   // a multiple of 8 blocks (XCDs)
#define HHG_P3(N, F) k_gs3d_planes<T, N, F><<<g, 512, 0, st>>>(lk, tb, u, uo, b, tiles, ntiles, sA)
    if (lk.n <= 16) { if (fine) HHG_P3(16, true); else HHG_P3(16, false); }
    else if (lk.n <= 32) { if (fine) HHG_P3(32, true); else HHG_P3(32, false); }
    else { if (fine) HHG_P3(64, true); else HHG_P3(64, false); }
#undef HHG_P3
    return true;
  }
  if (ntiles > 0) {
    // red-black with per-macro coefficient on a level with the plane-streaming tile table
    if (!rb) return false;
    const unsigned g = (unsigned)(((int64_t)lk.nmacro * ntiles + 7) / 8 * 8);   // a multiple of 8 blocks (XCDs)
    if (fine) k_gs3d_stream<T, true><<<g, 256, 0, st>>>(lk, tb, u, uo, b, tiles, ntiles, sA);
    else k_gs3d_stream<T, false><<<g, 256, 0, st>>>(lk, tb, u, uo, b, tiles, ntiles, sA);
    return true;
  }
  if (!itab || lk.n > kMacroLdsN) return false;
  const size_t shm = (size_t)lk.Sraw * sizeof(T);
  if (shm > 64 * 1024) return false;
  const unsigned blk = lk.NI >= 512 ? 1024 : 256;
#define HHG_F3(C, F) k_gs3d_macro<T, C, F><<<(unsigned)lk.nmacro, blk, shm, st>>>(lk, tb, u, b, itab, itab_off, rb, sA)
  if (rb) { if (fine) HHG_F3(2, true); else HHG_F3(2, false); }
  else { if (fine) HHG_F3(4, true); else HHG_F3(4, false); }
#undef HHG_F3
  return true;
}

template <typename T>
void launch_iface_tasks(int dim, const LK& lk, const Tables& tb, const int32_t* tp, const int32_t* tq, const int32_t* tco,
                        const int32_t* tseg, const int32_t* wmax, int w0, int w1, const T* xi, const T* xf, T* uout,
                        T* umirror, const T* b, int jacobi, double omega, double sA, hipStream_t st) {
  if (w1 <= w0) return;
  const unsigned g = grid8((w1 - w0 + 3) / 4);
  if (dim == 3)
    k_iface_tasks<3, T><<<g, 256, 0, st>>>(lk, tb, tp, tq, tco, tseg, wmax, w0, w1, xi, xf, uout, umirror, b, jacobi,
                                           omega, sA);
  else
    k_iface_tasks<2, T><<<g, 256, 0, st>>>(lk, tb, tp, tq, tco, tseg, wmax, w0, w1, xi, xf, uout, umirror, b, jacobi,
                                           omega, sA);
}

template <typename T>
void launch_iface_tasks_1wg(int dim, const LK& lk, const Tables& tb, const int32_t* tp, const int32_t* tq,
                            const int32_t* tco, const int32_t* tseg, const int32_t* wmax, const int32_t* woff, int c0,
                            int c1, const T* xi, const T* xf, T* uout, T* umirror, const T* b, double sA, bool pre,
                            hipStream_t st, int sweeps) {
  if (c1 <= c0) return;
  // preloading form: the caller has checked that every class has at most 16 wavefronts
  if (pre && c1 - c0 <= iface_pre_classes(dim, sizeof(T) == 8)) {
    if (dim == 3) {
      if constexpr (pre_classes<3, T>() > 0)
        k_iface_tasks_1wg_pre<3, T, pre_classes<3, T>()><<<1, 1024, 0, st>>>(lk, tb, tp, tq, tco, tseg, wmax, woff, c0,
                                                                             c1, xi, xf, uout, umirror, b, sA);
    } else {
      k_iface_tasks_1wg_pre<2, T, pre_classes<2, T>()><<<1, 1024, 0, st>>>(lk, tb, tp, tq, tco, tseg, wmax, woff, c0,
                                                                           c1, xi, xf, uout, umirror, b, sA);
    }
    return;
  }
  if (dim == 3)
    k_iface_tasks_1wg<3, T><<<1, 1024, 0, st>>>(lk, tb, tp, tq, tco, tseg, wmax, woff, c0, c1, xi, xf, uout, umirror, b,
                                                sA, sweeps);
  else
    k_iface_tasks_1wg<2, T><<<1, 1024, 0, st>>>(lk, tb, tp, tq, tco, tseg, wmax, woff, c0, c1, xi, xf, uout, umirror, b,
                                                sA, sweeps);
}

template <typename T>
void launch_smooth_iface(int dim, bool p1, const LK& lk, const Tables& tb, const int32_t* list, int count, const T* xi,
                         const T* xf, T* uout, T* umirror, const T* b, int jacobi, double omega, double sA,
                         const double* kn, hipStream_t st) {
  if (count <= 0) return;
  const unsigned g = nblk(count);
#define HHG_IF(D, P) \
  k_smooth_iface<D, T, P><<<g, 256, 0, st>>>(lk, tb, list, count, xi, xf, uout, umirror, b, jacobi, omega, sA, kn)
  if (dim == 3) {
    if (p1) HHG_IF(3, true); else HHG_IF(3, false);
  } else {
    if (p1) HHG_IF(2, true); else HHG_IF(2, false);
  }
#undef HHG_IF
}

template <typename T>
void launch_iface_sweep_1wg(int dim, bool p1, const LK& lk, const Tables& tb, const int32_t* list, const int32_t* coff,
                            int c0, int c1, const T* xi, const T* xf, T* uout, T* umirror, const T* b, double sA,
                            const double* kn, hipStream_t st) {
  if (c1 <= c0) return;
#define HHG_IW(D, P) \
  k_iface_sweep_1wg<D, T, P><<<1, 1024, 0, st>>>(lk, tb, list, coff, c0, c1, xi, xf, uout, umirror, b, sA, kn)
  if (dim == 3) {
    if (p1) HHG_IW(3, true); else HHG_IW(3, false);
  } else {
    if (p1) HHG_IW(2, true); else HHG_IW(2, false);
  }
#undef HHG_IW
}

template <typename Tin, typename Tout>
void launch_apply(int dim, bool p1, const LK& lk, const Tables& tb, const Tin* x, const Tin* b, Tout* y, int op,
                  double scale, double alpha, double beta, int zero_dir, const double* kn, hipStream_t st) {
  if (dim == 2 && !(p1 && op == 0)) {
    const int nseg = (lk.n + 1 + 61) / 62, nrb = (lk.n + 1 + kApplyRowsOp - 1) / kApplyRowsOp;
    const int nint = lk.nmacro * nrb * nseg;
    const int nbnd = (int)(((int64_t)lk.nmacro * 3 * lk.n + 63) / 64);
    const unsigned gw = (unsigned)(((int64_t)nint + nbnd + 3) / 4);
    k_apply2d_rows<Tin, Tout><<<gw, 256, 0, st>>>(lk, tb, x, b, y, op, scale, alpha, beta, zero_dir, nseg, nint);
    return;
  }
  if (dim == 3 && !(p1 && op == 0) && lk.n >= lk.rows3d_min) {
    const int nrows = (lk.n + 1) * (lk.n + 2) / 2;
    const int64_t waves = (int64_t)lk.nmacro * nrows;
    const unsigned gw = (unsigned)((waves + 31) / 32 * 8);   // 4 rows per block, a multiple of 8 blocks
    k_apply3d_rows<Tin, Tout><<<gw, 256, 0, st>>>(lk, tb, x, b, y, op, scale, alpha, beta, zero_dir, nrows);
    return;
  }
  const unsigned g = grid8((int64_t)lk.nmacro * ((lk.Sraw + 255) / 256));
  if (dim == 3) {
    if (p1) k_apply<3, Tin, Tout, true><<<g, 256, 0, st>>>(lk, tb, x, b, y, op, scale, alpha, beta, zero_dir, kn);
    else k_apply<3, Tin, Tout, false><<<g, 256, 0, st>>>(lk, tb, x, b, y, op, scale, alpha, beta, zero_dir, kn);
  } else {
    if (p1) k_apply<2, Tin, Tout, true><<<g, 256, 0, st>>>(lk, tb, x, b, y, op, scale, alpha, beta, zero_dir, kn);
    else k_apply<2, Tin, Tout, false><<<g, 256, 0, st>>>(lk, tb, x, b, y, op, scale, alpha, beta, zero_dir, kn);
  }
}

template <typename Tin, typename Tout>
void launch_iface_residual_tasks(int dim, const LK& lk, const Tables& tb, const int32_t* tp, const int32_t* tq,
                                 const int32_t* tco, const int32_t* tseg, const int32_t* wmax, int w0, int w1,
                                 const Tin* x, const Tin* b, Tout* y, double sA, hipStream_t st) {
  if (w1 <= w0) return;
  const unsigned g = grid8((w1 - w0 + 3) / 4);
  if (dim == 3)
    k_iface_residual_tasks<3, Tin, Tout><<<g, 256, 0, st>>>(lk, tb, tp, tq, tco, tseg, wmax, w0, w1, x, b, y, sA);
  else
    k_iface_residual_tasks<2, Tin, Tout><<<g, 256, 0, st>>>(lk, tb, tp, tq, tco, tseg, wmax, w0, w1, x, b, y, sA);
}
template void launch_iface_residual_tasks<double, float>(int, const LK&, const Tables&, const int32_t*, const int32_t*,
                                                         const int32_t*, const int32_t*, const int32_t*, int, int,
                                                         const double*, const double*, float*, double, hipStream_t);

template <typename Tin, typename Tout>
void launch_iface_residual(int dim, bool p1, const LK& lk, const Tables& tb, const Tin* x, const Tin* b, Tout* y,
                           double sA, const double* kn, hipStream_t st) {
  if (lk.nIface <= 0) return;
  const unsigned g = grid8(nblk(lk.nIface));
  if (dim == 3) {
    if (p1) k_iface_residual<3, Tin, Tout, true><<<g, 256, 0, st>>>(lk, tb, x, b, y, sA, kn);
    else k_iface_residual<3, Tin, Tout, false><<<g, 256, 0, st>>>(lk, tb, x, b, y, sA, kn);
  } else {
    if (p1) k_iface_residual<2, Tin, Tout, true><<<g, 256, 0, st>>>(lk, tb, x, b, y, sA, kn);
    else k_iface_residual<2, Tin, Tout, false><<<g, 256, 0, st>>>(lk, tb, x, b, y, sA, kn);
  }
}

template <typename T>
void launch_restrict(int dim, const LK& f, const LK& c, const Tables& tb, const T* rf, T* bc, hipStream_t st, T* zc) {
  if (dim == 2) {
    const int nseg = (c.n + 1 + kRestrictCols - 1) / kRestrictCols, nrb = (c.n + 1 + kRestrictRows - 1) / kRestrictRows;
    const unsigned gw = (unsigned)(((int64_t)c.nmacro * nrb * nseg + 3) / 4);
    k_restrict2d_rows<T><<<gw, 256, 0, st>>>(f, c, tb, rf, bc, zc, nseg);
    return;
  }
  const unsigned g = grid8((int64_t)c.nmacro * ((c.S + 255) / 256));
  if (dim == 3) k_restrict<3, T><<<g, 256, 0, st>>>(f, c, tb, rf, bc, zc);
  else k_restrict<2, T><<<g, 256, 0, st>>>(f, c, tb, rf, bc, zc);
}

template <typename T>
void launch_prolong(int dim, const LK& f, const LK& c, const Tables& tb, const T* ec, T* uf, T* w, const T* g, int mode,
                    hipStream_t st) {
  if (dim == 2) {
    const int nseg = (f.n + 1 + 63) / 64, nrb = (f.n + 1 + kApplyRows - 1) / kApplyRows;
    const unsigned gw = (unsigned)(((int64_t)f.nmacro * nrb * nseg + 3) / 4);
    k_prolong2d_rows<T><<<gw, 256, 0, st>>>(f, c, tb, ec, uf, w, g, mode, nseg);
    return;
  }
  const unsigned gr = grid8((int64_t)f.nmacro * ((f.Sraw + 255) / 256));
  if (dim == 3) k_prolong<3, T><<<gr, 256, 0, st>>>(f, c, tb, ec, uf, w, g, mode);
  else k_prolong<2, T><<<gr, 256, 0, st>>>(f, c, tb, ec, uf, w, g, mode);
}

void launch_inject(int dim, const LK& fine, const LK& coarse, const double* src, double* dst, hipStream_t st) {
  const unsigned g = (unsigned)(coarse.nmacro * ((coarse.Sraw + 255) / 256));
  const int shift = fine.l - coarse.l;
  if (dim == 3) k_inject<3><<<g, 256, 0, st>>>(fine, coarse, src, dst, shift);
  else k_inject<2><<<g, 256, 0, st>>>(fine, coarse, src, dst, shift);
}

void launch_init_dirichlet(int dim, const LK& lk, const Tables& tb, const double* g, double* x, double inner,
                           hipStream_t st) {
  const unsigned gr = (unsigned)(lk.nmacro * ((lk.Sraw + 255) / 256));
  if (dim == 3) k_init_dirichlet<3><<<gr, 256, 0, st>>>(lk, tb, g, x, inner);
  else k_init_dirichlet<2><<<gr, 256, 0, st>>>(lk, tb, g, x, inner);
}

template <typename T>
void launch_coarse(int n0, const int32_t* coff, const int64_t* copy, const double* Ainv, const T* rhs, T* x, int accumulate,
                   hipStream_t st) {
  if (n0 <= 0) return;
  // the explicit inverse serves n0 <= kCoarseDenseMax (16 KiB of LDS at most)
  k_coarse<T><<<nblk(n0), 256, (size_t)n0 * sizeof(double), st>>>(n0, coff, copy, Ainv, rhs, x, accumulate);
}

template <typename T>
void launch_coarse_factored(int n0, const int32_t* coff, const int64_t* copy, const int32_t* perm, const double* X,
                            double* scr, const T* rhs, T* x, int accumulate, hipStream_t st) {
  if (n0 <= 0) return;
  k_coarse_gather<T><<<nblk(n0), 256, 0, st>>>(n0, coff, copy, perm, rhs, scr);
  k_coarse_fwd<<<nblk(n0), 256, 0, st>>>(n0, X, scr, scr + n0);
  k_coarse_bwd<T><<<(unsigned)n0, 256, 0, st>>>(n0, X, scr + n0, coff, copy, perm, x, accumulate);
}
template void launch_coarse_factored<double>(int, const int32_t*, const int64_t*, const int32_t*, const double*,
                                             double*, const double*, double*, int, hipStream_t);
template void launch_coarse_factored<float>(int, const int32_t*, const int64_t*, const int32_t*, const double*,
                                            double*, const float*, float*, int, hipStream_t);

template <typename T>
void launch_dense_map(int rows, int ld, int kmax, const int32_t* gat, T* sum, const T* B, const T* b, int64_t nb,
                      const int32_t* off, const int32_t* copy, T* x, hipStream_t st) {
  if (rows <= 0) return;
  // table loads for the smallest bucket of copies per DoF that holds kmax
  if (kmax <= 8) k_dense_gather<T, 8><<<nblk(rows), 256, 0, st>>>(rows, kmax, gat, b, nb, sum);
  else if (kmax <= 16) k_dense_gather<T, 16><<<nblk(rows), 256, 0, st>>>(rows, kmax, gat, b, nb, sum);
  else if (kmax <= 32) k_dense_gather<T, 32><<<nblk(rows), 256, 0, st>>>(rows, kmax, gat, b, nb, sum);
  else k_dense_gather<T, kDenseMaxCopies><<<nblk(rows), 256, 0, st>>>(rows, kmax, gat, b, nb, sum);
  // 16 rows (wavefronts) per workgroup; LDS for the gathered b, rounded up to whole load groups
  const unsigned g = (unsigned)((rows + 15) / 16);
  const int qc = sizeof(T) == 4 ? 8 : 4, nqr = (ld / 256 + qc - 1) / qc * qc;
  k_dense_map<T><<<g, 1024, (size_t)nqr * 256 * sizeof(T), st>>>(rows, ld, B, sum, off, copy, x);
}
template void launch_dense_map<double>(int, int, int, const int32_t*, double*, const double*, const double*, int64_t,
                                       const int32_t*, const int32_t*, double*, hipStream_t);
template void launch_dense_map<float>(int, int, int, const int32_t*, float*, const float*, const float*, int64_t,
                                      const int32_t*, const int32_t*, float*, hipStream_t);

template <typename T>
void launch_unit(T* b, int64_t n, int64_t idx, hipStream_t st) {
  k_unit<T><<<nblk(n), 256, 0, st>>>(b, n, idx);
}
template void launch_unit<double>(double*, int64_t, int64_t, hipStream_t);
template void launch_unit<float>(float*, int64_t, int64_t, hipStream_t);

template <typename T>
void launch_dense_harvest(int rows, const int32_t* off, const int32_t* copy, int ld, int probe, const T* x, T* B,
                          hipStream_t st) {
  k_dense_harvest<T><<<nblk(rows), 256, 0, st>>>(rows, off, copy, ld, probe, x, B);
}
template void launch_dense_harvest<double>(int, const int32_t*, const int32_t*, int, int, const double*, double*,
                                           hipStream_t);
template void launch_dense_harvest<float>(int, const int32_t*, const int32_t*, int, int, const float*, float*,
                                          hipStream_t);

void launch_sqnorm(int dim, const LK& lk, const Tables& tb, const double* r, double* partial, double* out, hipStream_t st) {
  // 2D: one wavefront per row; 3D: one block per 256-entry chunk of a macro block
  const int64_t units = dim == 3 ? (int64_t)lk.nmacro * ((lk.Sraw + 255) / 256) : ((int64_t)lk.nmacro * (lk.n + 1) + 3) / 4;
  const unsigned g1 = (unsigned)(lk.NI > 0 ? std::min<int64_t>(kNormBlocks, units) : 0);
  const unsigned g2 = nblk(lk.nIface);
  if (g1) {
    if (dim == 3) k_sq_interior<3><<<g1, 256, 0, st>>>(lk, r, partial);
    else k_sq_interior<2><<<g1, 256, 0, st>>>(lk, r, partial);
  }
  if (g2) {
    if (dim == 3) k_sq_iface<3><<<g2, 256, 0, st>>>(lk, tb, r, partial + g1);
    else k_sq_iface<2><<<g2, 256, 0, st>>>(lk, tb, r, partial + g1);
  }
  k_sum<<<1, 256, 0, st>>>(partial, (int)(g1 + g2), out);
}

template <typename T>
void launch_sqnorm_closure(int dim, const LK& lk, const T* r, double* partial, double* out, hipStream_t st) {
  const int64_t chunks = (int64_t)lk.nmacro * ((lk.Sraw + 255) / 256);
  const unsigned g1 = (unsigned)std::min<int64_t>(kNormBlocks, chunks);
  if (dim == 3) k_sq_closure<3, T><<<g1, 256, 0, st>>>(lk, r, partial);
  else k_sq_closure<2, T><<<g1, 256, 0, st>>>(lk, r, partial);
  k_sum<<<1, 256, 0, st>>>(partial, (int)g1, out);
}
template void launch_sqnorm_closure<float>(int, const LK&, const float*, double*, double*, hipStream_t);

void launch_estimate(int dim, int norm, const LK& f, const LK& c, const Tables& tb, const double* u, const double* a,
                     const double* bc, double* partial, double* out, double scale, bool rows, hipStream_t st) {
  if (dim == 2 && norm == 0 && f.n >= 4 && rows) {
    const int nrb = (f.n - 2 + kEstRows - 1) / kEstRows, nseg = (f.n - 2 + 61) / 62, nbw = (3 * f.n + 63) / 64;
    const int wpm = nrb * nseg + nbw;
    const unsigned g = (unsigned)(((int64_t)f.nmacro * wpm + 3) / 4);
    k_estimate2d_rows<<<g, 256, 0, st>>>(f, c, tb, u, a, bc, partial, scale, nrb, nseg, nbw);
    k_macro_sum<<<(unsigned)(f.nmacro * 2), 256, 0, st>>>(partial, f.nmacro, wpm, 2, out);
    return;
  }
  const int nchunk = (int)((f.Sraw + 255) / 256);
  const unsigned g = (unsigned)(f.nmacro * nchunk);
#define HHG_EST(D, N) k_estimate<D, N><<<g, 256, 0, st>>>(f, c, tb, u, a, bc, partial, scale)
  if (dim == 3) {
    if (norm == 1) HHG_EST(3, 1); else if (norm == 2) HHG_EST(3, 2); else HHG_EST(3, 0);
  } else {
    if (norm == 1) HHG_EST(2, 1); else if (norm == 2) HHG_EST(2, 2); else HHG_EST(2, 0);
  }
#undef HHG_EST
  k_macro_sum<<<(unsigned)(f.nmacro * 2), 256, 0, st>>>(partial, f.nmacro, nchunk, 2, out);
}

void launch_bilinear(int dim, const LK& lk, const Tables& tb, const double* x, const double* y, double* partial,
                     double* out, double sA, hipStream_t st) {
  const int nchunk = (int)((lk.Sraw + 255) / 256);
  const unsigned g = (unsigned)(lk.nmacro * nchunk);
  if (dim == 3) k_bilinear<3><<<g, 256, 0, st>>>(lk, tb, x, y, partial, sA);
  else k_bilinear<2><<<g, 256, 0, st>>>(lk, tb, x, y, partial, sA);
  k_macro_sum<<<(unsigned)lk.nmacro, 256, 0, st>>>(partial, lk.nmacro, nchunk, 1, out);
}

void launch_canon_to_full(int dim, const LK& lk, const Tables& tb, const double* canon, double* full, int mode,
                          hipStream_t st) {
  const unsigned g = (unsigned)(lk.nmacro * ((lk.Sraw + 255) / 256));
  if (dim == 3) k_canon_to_full<3><<<g, 256, 0, st>>>(lk, tb, canon, full, mode);
  else k_canon_to_full<2><<<g, 256, 0, st>>>(lk, tb, canon, full, mode);
}

void launch_full_to_canon(int dim, const LK& lk, const Tables& tb, const double* full, double* canon, int mode,
                          hipStream_t st) {
  if (dim == 3) k_full_to_canon<3><<<nblk(lk.ndof), 256, 0, st>>>(lk, tb, full, canon, mode);
  else k_full_to_canon<2><<<nblk(lk.ndof), 256, 0, st>>>(lk, tb, full, canon, mode);
}

void launch_dof_coords(int dim, const LK& lk, const Tables& tb, const double* mxyz, const int32_t* cells, double* xyz,
                       hipStream_t st) {
  if (dim == 3) k_dof_coords<3><<<nblk(lk.ndof), 256, 0, st>>>(lk, tb, mxyz, cells, xyz);
  else k_dof_coords<2><<<nblk(lk.ndof), 256, 0, st>>>(lk, tb, mxyz, cells, xyz);
}

template <typename T>
void launch_fill(T* x, int64_t n, T v, hipStream_t st) {
  if (n > 0) k_fill<T><<<nblk(n), 256, 0, st>>>(x, n, v);
}
void launch_add_f32(double* u, const float* e, int64_t n, hipStream_t st) {
  if (n > 0) k_add_f32<<<nblk(n), 256, 0, st>>>(u, e, n);
}
void launch_copy(double* dst, const double* src, int64_t n, hipStream_t st) {
  if (n > 0) k_copy<<<nblk(n), 256, 0, st>>>(dst, src, n);
}

// explicit instantiations
template void launch_smooth_interior<double>(int, bool, const LK&, const Tables&, const double*, double*, const double*,
                                             int, int, int, double, double, const double*, bool, hipStream_t);
template void launch_smooth_interior<float>(int, bool, const LK&, const Tables&, const float*, float*, const float*, int,
                                            int, int, double, double, const double*, bool, hipStream_t);
template bool launch_gs_fused<double>(int, bool, const LK&, const Tables&, double*, double*, const double*,
                                      const int32_t*, int, const uint32_t*, const int32_t*, int, double, bool, hipStream_t,
                                      const double*, int, double*, bool);
template bool launch_gs_fused<float>(int, bool, const LK&, const Tables&, float*, float*, const float*, const int32_t*,
                                     int, const uint32_t*, const int32_t*, int, double, bool, hipStream_t, const float*,
                                     int, float*, bool);
template void launch_iface_tasks<double>(int, const LK&, const Tables&, const int32_t*, const int32_t*, const int32_t*,
                                         const int32_t*, const int32_t*, int, int, const double*, const double*, double*,
                                         double*, const double*, int, double, double, hipStream_t);
template void launch_iface_tasks<float>(int, const LK&, const Tables&, const int32_t*, const int32_t*, const int32_t*,
                                        const int32_t*, const int32_t*, int, int, const float*, const float*, float*,
                                        float*, const float*, int, double, double, hipStream_t);
template void launch_iface_tasks_1wg<double>(int, const LK&, const Tables&, const int32_t*, const int32_t*,
                                             const int32_t*, const int32_t*, const int32_t*, const int32_t*, int, int,
                                             const double*, const double*, double*, double*, const double*, double, bool,
                                             hipStream_t, int);
template void launch_iface_tasks_1wg<float>(int, const LK&, const Tables&, const int32_t*, const int32_t*,
                                            const int32_t*, const int32_t*, const int32_t*, const int32_t*, int, int,
                                            const float*, const float*, float*, float*, const float*, double, bool,
                                            hipStream_t, int);
template void launch_smooth_iface<double>(int, bool, const LK&, const Tables&, const int32_t*, int, const double*,
                                          const double*, double*, double*, const double*, int, double, double,
                                          const double*, hipStream_t);
template void launch_smooth_iface<float>(int, bool, const LK&, const Tables&, const int32_t*, int, const float*,
                                         const float*, float*, float*, const float*, int, double, double, const double*,
                                         hipStream_t);
template void launch_iface_sweep_1wg<double>(int, bool, const LK&, const Tables&, const int32_t*, const int32_t*, int,
                                             int, const double*, const double*, double*, double*, const double*, double,
                                             const double*, hipStream_t);
template void launch_iface_sweep_1wg<float>(int, bool, const LK&, const Tables&, const int32_t*, const int32_t*, int, int,
                                            const float*, const float*, float*, float*, const float*, double,
                                            const double*, hipStream_t);
template void launch_apply<double, double>(int, bool, const LK&, const Tables&, const double*, const double*, double*,
                                           int, double, double, double, int, const double*, hipStream_t);
template void launch_apply<double, float>(int, bool, const LK&, const Tables&, const double*, const double*, float*, int,
                                          double, double, double, int, const double*, hipStream_t);
template void launch_apply<float, float>(int, bool, const LK&, const Tables&, const float*, const float*, float*, int,
                                         double, double, double, int, const double*, hipStream_t);
template void launch_iface_residual<double, float>(int, bool, const LK&, const Tables&, const double*, const double*,
                                                  float*, double, const double*, hipStream_t);
template void launch_iface_residual<double, double>(int, bool, const LK&, const Tables&, const double*, const double*,
                                                   double*, double, const double*, hipStream_t);
template void launch_restrict<double>(int, const LK&, const LK&, const Tables&, const double*, double*, hipStream_t,
                                      double*);
template void launch_restrict<float>(int, const LK&, const LK&, const Tables&, const float*, float*, hipStream_t, float*);
template void launch_prolong<double>(int, const LK&, const LK&, const Tables&, const double*, double*, double*,
                                     const double*, int, hipStream_t);
template void launch_prolong<float>(int, const LK&, const LK&, const Tables&, const float*, float*, float*, const float*,
                                    int, hipStream_t);
template void launch_coarse<double>(int, const int32_t*, const int64_t*, const double*, const double*, double*, int,
                                    hipStream_t);
template void launch_coarse<float>(int, const int32_t*, const int64_t*, const double*, const float*, float*, int,
                                   hipStream_t);
template void launch_fill<double>(double*, int64_t, double, hipStream_t);
template void launch_fill<float>(float*, int64_t, float, hipStream_t);

void launch_impose_dirichlet(int dim, const LK& lk, const Tables& tb, const double* g, double* x, hipStream_t st) {
  const unsigned gr = (unsigned)(lk.nmacro * ((lk.Sraw + 255) / 256));
  if (dim == 3) k_impose_dirichlet<3><<<gr, 256, 0, st>>>(lk, tb, g, x);
  else k_impose_dirichlet<2><<<gr, 256, 0, st>>>(lk, tb, g, x);
}

void launch_transfer(int dim, const LK& fn, const double* mxyz_new, const LK& fo, const double* mxyz_old,
                     const int32_t* coff, const int32_t* cand, const double* uold, double* unew, hipStream_t st) {
  const unsigned gr = (unsigned)(fn.nmacro * ((fn.Sraw + 255) / 256));
  if (dim == 3) k_transfer3d<<<gr, 256, 0, st>>>(fn, mxyz_new, fo, mxyz_old, coff, cand, uold, unew);
  else k_transfer2d<<<gr, 256, 0, st>>>(fn, mxyz_new, fo, mxyz_old, coff, cand, uold, unew);
}

}  // namespace hhg
