// Internal declarations of the HHG library: lattice geometry of a refined macro element,
// the per-context plan, and the kernel launch interface.
//
// Lattice of one macro element refined to level l (n = 2^l micro intervals per edge): the
// micro nodes are the points x0 + (i/n)(x1-x0) + (j/n)(x2-x0) [+ (k/n)(x3-x0)] with integer
// barycentric coordinates c = (n-i-j-k, i, j, k) >= 0.  Uniform refinement (the 4-split in
// 2D, Bey's rule in 3D) produces the lattice triangulation whose edges run along
//   2D: +-{e1, e2, e2-e1}
//   3D: +-{e1, e2, e3, e2-e1, e3-e1, e3-e2, e1-e2+e3}
// (in 3D, with p = (i, i+j, i+j+k) it is the Kuhn triangulation of the unit-cube lattice).
// Every vector of a level is stored per macro over its whole closure, in the order
//   3D: slab k (outer), row j, index i (inner);   2D: row j (outer), index i (inner),
// padded to a multiple of 64 entries per macro.  DoFs on macro vertices, edges and faces are
// therefore stored once per adjacent macro (ghost copies).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "hhg.h"

namespace hhg {

constexpr int kMaxMask = 16;   // zero-set masks of the barycentric coordinates (bit q: c_q == 0)
constexpr int kNDir3 = 15, kNDir2 = 7;
constexpr int kNType3 = 6, kNType2 = 2;
// fused interior sweeps: a 2D tile is (64 - 2 C) columns (one wavefront) x tile_rows(C, n) rows
// (C = interior colours).  A wavefront sweeps its tile's rows one after another, so the height
// sets both the length of its chain and the number of workgroups of a launch: short tiles up to
// n = kShortTileMaxN (latency-bound levels), taller ones above.  Multicolour heights are
// multiples of 3, so every tile starts on a row = 1 (mod 3).
constexpr int kShortTileMaxN = 128;
constexpr int tile_rows(int C, int n) {
  return C == 3 ? (n <= kShortTileMaxN ? 6 : 18) : (n <= kShortTileMaxN ? 8 : 16);
}
// the largest 3D macro level kept whole in LDS
constexpr int kMacroLdsN = 32;
// plane-streaming 3D red-black sweep: a tile holds kS3I x kS3J interior points of a plane and
// streams kS3K planes; LDS planes are 64 x (kS3J + 4) points (two-point halo in i and j)
constexpr int kS3I = 60, kS3J = 28, kS3K = 32;
constexpr int kStream3dMinN = 256;  // levels with n >= this use it (red-black, per-macro coefficient)
// whole-plane 3D red-black sweep: levels with kPlane3dMinN <= n <= kPlane3dMaxN (a plane of the
// closure fits one LDS slot and a pair of interior rows one wavefront; below n = 64 the LDS
// macro sweep measured faster); the interior planes of a macro are cut into chunks so that a
// level has about kPlane3dBlocks workgroups
constexpr int kPlane3dMinN = 64, kPlane3dMaxN = 64, kPlane3dBlocks = 2048;
// levels whose largest interface colour class has at most this many DoFs sweep all interface
// classes in one single-workgroup launch
constexpr int kIfaceOneGroup = 4096;
// lane-parallel interface sweeps: levels whose largest class spans at most this many
// wavefronts sweep all classes in one workgroup of 16 wavefronts
constexpr int kTaskOneGroupWaves = 32;
// record of one 2D macro edge for the edge-class sweep (int32 words): [0] copies | Dirichlet
// << 2; per copy k at 2 + kEdgeCopyWords k: macro, slot of the edge's lower-id vertex | slot
// of its higher-id vertex << 8 | zero-set mask << 16, then the macro's coefficient and its 7
// unit stencil weights for that mask (doubles, words 2..17), then the mask's valid directions
constexpr int kEdgeCopyWords = 20;
constexpr int kEdgeRecWords = 2 + 2 * kEdgeCopyWords;
// level 0 is solved by its explicit inverse up to this many inner vertices, above it by the
// factored form (envelope Cholesky after reverse Cuthill-McKee)
constexpr int kCoarseDenseMax = 2048;
// dense map of the cycle on one coarse level k (the V-cycle of levels k .. 0 from a zero
// iterate, as one matrix from the assembled right-hand side to the iterate): at most this many
// rows and columns (inner DoFs of level k) and bytes (the float32 and float64 maps together)
constexpr int kDenseMaxRows = 8192, kDenseMaxCopies = 64;
constexpr int64_t kDenseMaxBytes = 512ll << 20;
// blocks of the interior part of a squared norm (one partial each)
constexpr int kNormBlocks = 8192;
// interior rows per wavefront of the 2D row estimator
constexpr int kEstRows = 4;

// direction tables: index 0 is the centre, 1..H positive, H+1..2H negative
constexpr int kDir3[7][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {-1, 1, 0}, {-1, 0, 1}, {0, -1, 1}, {1, -1, 1}};
constexpr int kDir2[3][2] = {{1, 0}, {0, 1}, {-1, 1}};

// A macro-primitive incidence: macro `macro` contains the primitive; slot[r] is the local
// vertex slot (0..dim) of the primitive's r-th vertex (sorted by global id); mask has bit q
// set for every local slot q that is not a vertex of the primitive.
struct Inc {
  int32_t macro;
  uint8_t slot[3];
  uint8_t mask;
};

// Device-side tables, all living inside the bound workspace.
struct Tables {
  int dim = 0;
  int nmacro = 0;
  int nV = 0, nE = 0, nF = 0;          // primitive counts
  const double* stiff = nullptr;       // [nmacro][16][ndir] unit-coefficient stiffness, n = 1 scale
  const double* mass = nullptr;        // [nmacro][16][ndir] mass, n = 1 scale
  const double* elemK = nullptr;       // [nmacro][ntype][(d+1)^2] unit element stiffness, n = 1 scale
  const double* kappa = nullptr;       // [nmacro]
  const int32_t* subprim = nullptr;    // [nmacro][16] global primitive id of the sub-primitive with that zero-set
  const uint8_t* suborder = nullptr;   // [nmacro][16] slots of that primitive sorted by global id, 2 bits each
  const uint16_t* dirbits = nullptr;   // [nmacro] bit `mask` set: that sub-primitive is Dirichlet
  const uint16_t* ownbits = nullptr;   // [nmacro] bit `mask` set: this macro is the lowest-id owner
  const int32_t* rbpar = nullptr;      // [nmacro][4] red-black parity: x0 parity at level scale factor, s1, s2, s3
  const int32_t* inc_off = nullptr;    // [nprim+1] CSR offsets into inc
  const Inc* inc = nullptr;            // incidences, macro id ascending per primitive
  const uint8_t* primdir = nullptr;    // [nprim] primitive is Dirichlet
  uint16_t validdirs[kMaxMask] = {};   // per zero-set mask: directions whose neighbour is in the closure
  uint32_t incvalid[kMaxMask] = {};    // per zero-set mask: incident (type, vertex) pairs inside the macro
};

// Per-level layout and buffers.
struct Level {
  int l = 0, n = 1;
  int64_t Sraw = 0, S = 0;      // closure entries per macro (raw / padded)
  int64_t NI = 0;               // macro-interior DoFs per macro
  int64_t nEd = 0, nFd = 0;     // DoFs interior to one edge / one face
  int64_t nIface = 0;           // DoFs on vertices, edges, faces (canonical prefix)
  int64_t ndof = 0;             // canonical DoF count
  int64_t nfull = 0;            // nmacro * S
  int ncolours = 0;             // colours used by the Gauss-Seidel sweep
  int interior_colours = 0;     // colours present among macro-interior DoFs
  std::vector<int64_t> interior_per_colour;   // macro-interior DoFs of each colour (all macros)
  std::vector<int32_t> colour_off;     // host: CSR offsets of the interface colour lists
  std::vector<int32_t> colour_list;    // host: interface DoF ids per colour (non-Dirichlet)
  // device buffers (inside workspace)
  double *x = nullptr, *t = nullptr, *bf = nullptr, *rc = nullptr, *g = nullptr, *w = nullptr, *kn = nullptr;
  float *x32 = nullptr, *t32 = nullptr, *b32 = nullptr;
  double* x2 = nullptr;                // second iterate buffer of the out-of-place 2D fused sweep
  float* x2_32 = nullptr;
  int32_t* d_colour_list = nullptr;
  int32_t* d_colour_off = nullptr;
  int max_iface_class = 0;
  // lane-parallel interface sweep (Gauss-Seidel, per-macro coefficient): one lane per
  // (interface DoF, incident macro), lanes of one DoF consecutive in a wavefront; arrays of
  // 64 entries per wavefront, wavefronts of class c are task_woff[c] .. task_woff[c+1]-1.
  // Per lane: task_copy = level-vector index of the copy (-1: padding lane), task_info =
  // macro | zero-set mask << 24 | Dirichlet << 28, task_loc = i | j << 11 | k << 22 (closure
  // coordinates in the macro), task_seg = first lane of the DoF | lane count << 8.
  bool task_ok = false;
  std::vector<int32_t> task_copy, task_info, task_loc, task_seg, task_wmax, task_woff;
  int32_t *d_task_copy = nullptr, *d_task_info = nullptr, *d_task_loc = nullptr, *d_task_seg = nullptr,
          *d_task_wmax = nullptr, *d_task_woff = nullptr;
  int64_t off_tcopy = 0, off_tinfo = 0, off_tloc = 0, off_tseg = 0, off_twmax = 0, off_twoff = 0;
  // 2D edge classes in one launch (k_iface2d_edges, from the context's edge records):
  // dvcopy = level-vector indices of the copies of Dirichlet vertices (which the same launch
  // copies); the vertex classes c_vr0 .. ncolours - 1 follow (wheels or interface tasks)
  bool fused_iface = false;
  int c_vr0 = 0;
  std::vector<int32_t> dvcopy;
  int32_t* d_dvcopy = nullptr;
  int64_t off_dvcopy = 0;
  // vertex classes by wheels (k_iface2d_wheels): one lane per DoF copy, 64 per wavefront;
  // wh_info = macro | mask << 24 | (class - c_vr0) << 28, wh_loc = i | j << 11, wh_seg = lead
  // lane | copies << 8, wh_src = two words per lane with the lane of each direction's
  // neighbour (8 bits per direction 1..4, then 5..6; 0xff: from memory), wh_wmax per wavefront
  bool wheels = false;
  std::vector<int32_t> wh_copy, wh_info, wh_loc, wh_seg, wh_src, wh_wmax;
  std::vector<double> wh_cw;          // per lane: kappa, then the 7 unit weights (struct of arrays)
  int32_t *d_whcopy = nullptr, *d_whinfo = nullptr, *d_whloc = nullptr, *d_whseg = nullptr, *d_whsrc = nullptr,
          *d_whwmax = nullptr;
  double* d_whcw = nullptr;
  // wheels in the launch of the edge classes: per lane the edge-class neighbour to recompute,
  // e | side << 24 | direction << 25 (side 1: a = n - 2 on the edge, else a = 2), or -1
  bool wh_merge = false;
  std::vector<int32_t> wh_e2;
  int32_t* d_whe2 = nullptr;
  int64_t off_whe2 = 0;
  // and that neighbour's rows, 16 entries per lane (struct of arrays): per copy k of it,
  // wh_a2i[8k] its closure index (-1: none), [8k + dd] the neighbour in direction dd (-1:
  // none), [8k + 7] bit dd - 1 set for an interface neighbour; wh_a2w[8k] the coefficient
  // (filled in at upload), [8k + 1 + d] the unit stencil weight d
  std::vector<int32_t> wh_a2i;
  std::vector<double> wh_a2w;
  int32_t* d_wha2i = nullptr;
  double* d_wha2w = nullptr;
  int64_t off_wha2i = 0, off_wha2w = 0;
  int64_t off_whcopy = 0, off_whinfo = 0, off_whloc = 0, off_whseg = 0, off_whsrc = 0, off_whwmax = 0,
          off_whcw = 0;
  std::vector<int32_t> tiles;          // 2D: interior tiles (ti | tj << 16) of the fused sweep
  bool planes3d = false;               // 3D: tiles are plane chunks (k0 | k1 << 16) of k_gs3d_planes
  std::vector<uint32_t> itab;          // 3D, n <= kMacroLdsN: interior points (i | j << 10 | k << 20)
  int32_t* d_tiles = nullptr;
  uint32_t* d_itab = nullptr;
  std::vector<int32_t> itab_off;       // 3D: colour offsets of itab per parity pattern
  int32_t* d_itab_off = nullptr;
  int64_t off_itoff = 0;
  int64_t off_x = 0, off_t = 0, off_bf = 0, off_rc = 0, off_g = 0, off_w = 0, off_kn = -1, off_x32 = 0, off_t32 = 0,
          off_b32 = 0, off_cl = 0, off_tiles = 0, off_itab = 0, off_x2 = 0, off_x2_32 = 0, off_coff = 0;
};

}  // namespace hhg

// The opaque context.
struct hhg_ctx_s {
  int dim = 0, L = 0;
  hhg_options opt{};
  int64_t nV = 0, nC = 0;
  std::vector<double> coords;       // nV * dim
  std::vector<int32_t> cells;       // nC * (dim+1)
  std::vector<double> kappa_cell;   // nC
  std::vector<uint8_t> vdir_user;   // per vertex (empty = whole boundary)
  int dyadic_p = 0;                 // smallest p with coords * 2^p integral (-1: not dyadic)

  // primitives (host)
  std::vector<int32_t> edges;       // nE * 2 sorted
  std::vector<int32_t> faces;       // nF * 3 sorted
  int nE = 0, nF = 0;
  std::vector<uint8_t> primdir;     // nprim
  std::vector<int32_t> inc_off;     // nprim + 1
  std::vector<hhg::Inc> inc;
  std::vector<int32_t> subprim;     // nC * 16
  std::vector<uint8_t> suborder;    // nC * 16
  std::vector<uint16_t> dirbits, ownbits;
  std::vector<int32_t> rbpar;       // nC * 4
  std::vector<double> stiff, mass, elemK;
  std::vector<int32_t> erec;        // 2D edge records of the edge-class sweep (kEdgeRecWords per edge)
  std::vector<uint16_t> validdirs;  // [16] bitmask of valid directions per zero-set mask
  std::vector<uint32_t> incvalid;   // [16] bitmask of valid incident (type, vertex) pairs

  // coarse (level 0) solve
  int n0 = 0;                       // inner coarse vertices
  std::vector<int32_t> coarse_vertex;      // inner vertex ids
  std::vector<int32_t> coarse_copy_off;    // CSR into coarse_copy
  std::vector<int64_t> coarse_copy;        // full-layout indices at level 0
  std::vector<double> Ainv;                // n0 * n0: the inverse, or X = L^{-1} (factored form)
  bool coarse_factored = false;            // n0 > kCoarseDenseMax: x = P^T X^T X P r
  std::vector<int32_t> coarse_perm;        // position -> inner vertex (reverse Cuthill-McKee)

  std::vector<hhg::Level> lev;
  hhg::Tables tab;

  // workspace
  size_t ws_bytes = 0;
  char* ws = nullptr;
  void* stream = nullptr;
  bool bound = false;
  bool solved = false;              // the FMG level solutions of the last solve are valid
  bool have_u = false;              // u_L of the last solve is valid (FMG or cycles)
  bool kappa_nodal_set = false;
  // workspace offsets of tables
  int64_t o_stiff = 0, o_mass = 0, o_elemK = 0, o_kappa = 0, o_subprim = 0, o_suborder = 0, o_dirbits = 0,
          o_ownbits = 0, o_rbpar = 0, o_incoff = 0, o_inc = 0, o_primdir = 0, o_ccopyoff = 0, o_ccopy = 0,
          o_ainv = 0, o_red = 0, o_scal = 0, o_mxyz = 0, o_aux0 = 0, o_aux1 = 0, o_erec = 0, o_cperm = 0, o_cscr = 0;
  int64_t red_capacity = 0;         // doubles in the reduction scratch
  double* d_red = nullptr;          // reduction scratch
  double* d_scal = nullptr;         // small scalar scratch
  int32_t* d_ccopy_off = nullptr;
  int64_t* d_ccopy = nullptr;
  double* d_ainv = nullptr;
  int32_t* d_cperm = nullptr;       // factored level 0: permutation, and two n0 scratch vectors
  double* d_cscr = nullptr;
  double* d_aux0 = nullptr;         // level-L scratch: the recomputed solution inside hhg_adjoint
  double* d_aux1 = nullptr;         // level-L scratch: reference iterate of the residual norm

  bool static_ws = false;           // bound to the library's static workspace (no graphs, no events)
  int static_dev = -1;              // device whose static workspace this context holds (-1: none)
  void* ev0 = nullptr;              // hipEvent_t pair for timing
  void* ev1 = nullptr;
  int last_nu = 0;                  // FMG parameters of the last solve (estimator needs L >= 2)
  std::vector<double> res_hist;     // relative residual after each extra cycle of the last solve
  // per-launch timing of the finest-level interior smoother (hhg_bench_smoother)
  std::vector<void*> prof_ev;       // hipEvent_t pairs
  int prof_used = 0;
  bool prof_on = false;
  bool no_fused = false;            // force class-by-class interior launches (testing)
  bool no_tasks = false;            // force the per-DoF interface kernels (testing)
  // HIP graphs of the launch-bound sequences (FMG body; one extra cycle with its residual
  // norm), recorded once per parameter set on a private capture stream and replayed on the
  // caller's stream; key = kind | nu << 4 | pre << 12 | post << 20 | precision << 28 |
  // xswap << 32, key2 = the number of fixed extra cycles (kind 4)
  bool no_graph = false;            // run every launch eagerly (testing)
  bool no_preload = false;          // single-workgroup interface sweep without preloading (testing)
  bool force_rows3d = false;        // 3D row kernels at every level (testing)
  bool force_stream3d = false;      // 3D plane-streaming sweep from n = 4 on (testing)
  bool no_planes3d = false;         // no whole-plane 3D sweep (testing, timing)
  bool force_planes3d = false;      // whole-plane 3D sweep from n = 16 on (testing)
  bool two_launch_iface = false;    // 2D edge and vertex classes in two launches (testing, timing)
  bool generic_est = false;         // 2D L2 estimate by the one-thread-per-node kernel (testing)
  bool no_dense = false;            // no dense map of the coarse cycle (testing, timing)
  bool no_pro = false;              // cycle prolongation as its own launch (testing, timing)
  bool force_dense = false;         // dense map on the largest level that fits, up to L - 1 (testing)
  // dense map of the cycle on level dense_k: row and column r are inner DoF r of that level
  // (canonical order), with its copies dense_copy[dense_off[r] .. dense_off[r+1]) (level-vector
  // indices); dense_ld = rows rounded up to 256.  dense_key[p] = pre | post << 16 of the map
  // built for precision p (-1: none)
  // dense_gat[q * rows + r] = index + 1 of copy q of row r (0: none), q < dense_kmax; d_dsum
  // holds the gathered right-hand side of one product
  int dense_k = -1;
  int dense_rows = 0, dense_ld = 0, dense_kmax = 0;
  std::vector<int32_t> dense_off, dense_copy, dense_gat;
  int64_t o_dense32 = 0, o_dense64 = 0, o_doff = 0, o_dcopy = 0, o_dgat = 0, o_dsum = 0;
  float* d_dense32 = nullptr;
  double* d_dense64 = nullptr;
  int32_t *d_doff = nullptr, *d_dcopy = nullptr, *d_dgat = nullptr;
  void* d_dsum = nullptr;
  int64_t dense_key[2] = {-1, -1};
  bool dense_building = false;      // the map's own probe cycles run the ordinary path
  bool classwise_iface = false;     // 2D interface classes one launch each (testing)
  uint32_t xswap = 0;               // bit l (+16 for float32): level l's iterate is in its second buffer
  void* cap_stream = nullptr;       // hipStream_t used only while recording
  bool capturing = false;
  struct Recorded {
    int64_t key, key2;              // launch sequence and parameters (graph_key), extra count
    void* exec;                     // hipGraphExec_t
  };
  std::vector<Recorded> graphs;
  double prof_bytes = 0.0;

  std::string err;
};

namespace hhg {

// host setup (hhg_setup.cpp)
hhg_status build_topology(hhg_ctx c);
hhg_status build_stencils(hhg_ctx c);
hhg_status build_colouring(hhg_ctx c);
hhg_status build_coarse(hhg_ctx c, const double* kappa_vertex /* nullable, per vertex */);
void build_dense_plan(hhg_ctx c);
void plan_workspace(hhg_ctx c);
void fill_kappa_tables(hhg_ctx c);

// index helpers shared by host code
int64_t tet_count(int64_t m);
int64_t tri_count(int64_t m);
int64_t lin_closure(int dim, int n, int i, int j, int k);
int zero_mask(int dim, int n, int i, int j, int k);
// canonical DoF index of closure point (i,j,k) of macro m on level with n = 2^l
int64_t canonical_index(hhg_ctx c, const Level& lv, int m, int i, int j, int k);

}  // namespace hhg
