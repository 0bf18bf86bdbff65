// Internal declarations of the immersed-boundary library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ib.h"

namespace ib {

constexpr int kMaxOrder = 8;           // largest space order M supported
constexpr int kMaxTerms = 165;         // binomial(8+3, 3)
constexpr int kMaxRadiusCode = 40;     // radius codes 2r = 1..40 (r <= 20 cells)
constexpr int kMaxOps = 8;             // boundary-condition rows per boundary point
constexpr int kMaxOpTerms = 48;        // derivative terms per boundary-condition row
// depth columns of the 3D support balls taken by the LDS-tiled patch (radius 4.5 and 4)
constexpr int kColumns9 = 69, kColumns8 = 49;
constexpr int32_t kNoColumn = -1;
constexpr int kColPad = 16;            // entries after the last column-run record

void set_error(const char *fmt, ...);
ib_status hip_fail(hipError_t e, const char *what, const char *file, int line);

#define IB_HIP(call)                                                          \
  do {                                                                        \
    hipError_t _e = (call);                                                   \
    if (_e != hipSuccess) return ib::hip_fail(_e, #call, __FILE__, __LINE__); \
  } while (0)

// Device allocation that reports IB_ERR_OOM.
ib_status dalloc(void **p, size_t bytes);
template <class T>
ib_status dalloc_t(T **p, size_t count) {
  return dalloc(reinterpret_cast<void **>(p), count * sizeof(T));
}
void dfree(void *p);

// Lattice points of the ball |o| <= code/2 in memory order (z slowest, x fastest),
// packed as signed bytes (dx, dy, dz, 0); the same list for every grid.
struct BallTables {
  std::vector<int32_t> packed;             // all codes concatenated
  int start[kMaxRadiusCode + 2] = {0};
  int count[kMaxRadiusCode + 2] = {0};
  void build(int ndim, int max_code);
};

// Derivative operators of the boundary conditions, as sums of d^beta terms.
struct OpTerm {
  int8_t beta[3];
  int8_t normal_axis;   // -1: plain coefficient; else multiplied by normal[normal_axis]
  int8_t scaled;        // 1: also multiplied by the boundary point's mixed-surface coefficient
  double coef;
};
struct OpSet {
  int nops;
  int nterms[kMaxOps];
  OpTerm term[kMaxOps][kMaxOpTerms];
};
OpSet make_ops(int surface, int Mb, int ndim);
OpSet make_vops(int surface, int Mb, int ndim, int axis);
void add_laplacian_power(OpSet &ops, int slot, int q, int ndim, int normal_axis, int scaled = 0);
std::vector<int32_t> shifted_ball(int ndim, int code, const double shift[3]);
void staggered_first_derivative_weights(int M, double *w);   // offsets -(M-1)/2..(M-1)/2

// One family of modified staggered operators solved by the batched FP64 kernel.
struct FamilySpec {
  int family = 1;              // 1: d/dx_g of p at v_g nodes; 2: div v at p nodes
  int gaxis = 0;               // family 1: derivative axis (0 x, 1 y, 2 z)
  int nfields = 1, nblocks = 1;
  const uint8_t *fcls[3] = {nullptr, nullptr, nullptr};   // data-field classes
  double foff[3][3] = {{0}};   // node offset of each data field (half cells)
  int fblock[3] = {0, 0, 0};
  int baxis[3] = {0, 0, 0};    // family 2: velocity axis of each block
  double x0off[3] = {0, 0, 0}; // expansion point relative to the anchor node
  const uint8_t *xcls[3] = {nullptr, nullptr, nullptr};
  std::vector<int64_t> anchors;   // anchor nodes (memory order)
};
struct FamilyPoint {
  int k = 0, Mb = 0;
  std::vector<int32_t> field;  // per weight: data field
  std::vector<int32_t> off;    // per weight: packed lattice offset (dx, dy, dz)
  std::vector<double> w;
};


int n_terms(int M, int ndim);
void multi_indices(int M, int ndim, std::vector<int8_t> &out);   // [nterms][3]
void second_derivative_weights(int M, double *w);                 // offsets -M/2..M/2

}  // namespace ib

struct ib_weights;
namespace ib {
ib_status upload_ball_tables(ib_weights *w, hipStream_t st);
ib_status build_dense_records(ib_weights *w, hipStream_t st);
ib_status build_column_records(ib_weights *w, hipStream_t st);
ib_status solve_family(ib_weights *w, const FamilySpec &F, const int64_t *col_off_dev, hipStream_t st,
                       std::vector<FamilyPoint> &out);
}

struct ib_weights {
  int device = 0;
  int ndim = 3;
  int64_t nx = 1, ny = 1, nz = 1, N = 0;
  double h = 1.0;
  ib_params prm{};
  int M = 8;
  int64_t pitch = 0;               // padded x extent of the state's wavefields
  // geometry (device)
  double *Hs = nullptr;            // heights in grid units [ny][nx]
  uint8_t *node_class = nullptr;   // [N]
  int64_t nb = 0;
  double *bp = nullptr;            // [nb][8]: host x,y,z, x_b x,y,z, (normal kept below)
  double *bp_normal = nullptr;     // [nb][3]
  // IB points (device)
  int64_t nib = 0;
  int64_t *ib_node = nullptr;      // memory-order node index [nib]
  int16_t *ib_xyz = nullptr;       // [nib][4] x, y, z, radius code
  int32_t *ib_meta = nullptr;      // [nib][4] k, Mb, nw, woff
  double *ib_sigma = nullptr;      // [nib]
  int64_t sumw = 0;
  double *w64 = nullptr;           // [sumw]
  // stencil records used by the patch kernels: per point, the data-membership bit mask
  // of its support ball followed by the weights, in 32-bit units.
  uint32_t *rec32 = nullptr;
  uint32_t *rec64 = nullptr;
  uint32_t *rec_off32 = nullptr;   // [nib] offsets in 32-bit units
  uint32_t *rec_off64 = nullptr;
  int64_t rec32_words = 0, rec64_words = 0;
  // dense-range records (weights of every ball lattice point between the first and the
  // last data point of each support, zero where not data)
  float *dense32 = nullptr;
  double *dense64 = nullptr;
  int32_t *dense_first = nullptr, *dense_count = nullptr;
  uint32_t *dense_off = nullptr;
  int64_t dense_words = 0;
  // column-run records of the 3D supports of radius 4 and 4.5 (build_column_records):
  // first data plane per grid column, packed column tables (code 9 then code 8: dx, dy,
  // zr), per-point entry offsets and counts (-1: other supports), entries FP32 and FP64
  int16_t *zfirst = nullptr;
  int32_t *col_tab = nullptr;
  uint32_t *col_off = nullptr;
  int32_t *col_cnt = nullptr;
  float *col32 = nullptr;
  double *col64 = nullptr;
  int64_t col_words = 0;
  int32_t *ball = nullptr;         // packed ball tables
  int32_t *ball_meta = nullptr;    // [code][2] start, count (device)
  ib::BallTables balls;
  // first-order (pressure-velocity) form
  int form = 0;
  uint8_t *vcls[3] = {nullptr, nullptr, nullptr};   // classes of the v_n nodes
  std::vector<int32_t> pv_row_fam;    // per modified row: 0..ndim-1 gradient along that axis
                                      // (row node is a v node), ndim divergence (p node)
  std::vector<int64_t> pv_row_node;   // memory-order node index of the row
  std::vector<int64_t> pv_row_start;  // [nrows + 1]
  std::vector<int32_t> pv_ent_field;  // -1 p, n: v_n
  std::vector<int64_t> pv_ent_node;
  std::vector<double> pv_ent_w;
  int64_t pv_stats[4] = {0, 0, 0, 0};
  int max_code = 0;
  ib_stats stats{};
  // transposed IB rows for the adjoint, built on first use (-1: not built): receiving
  // nodes (padded index), run offsets [nj + 1], IB point and weight of each entry
  int64_t adj_nj = -1;
  uint32_t *adj_jnode = nullptr, *adj_joff = nullptr, *adj_jsrc = nullptr;
  float *adj_jw32 = nullptr;
  double *adj_jw64 = nullptr;
  // weights of the boundary-condition values (kept on request, second-order form): the
  // entries of IB point i are bc_off[i] .. bc_off[i] + bc_cnt[i] - 1, each
  // (boundary point << 3 | condition q) with its FP64 weight (grid units)
  int64_t nbc = 0;
  int bc_nq = 0;                   // conditions of the hierarchy at full order
  int64_t *bc_off = nullptr;
  int32_t *bc_cnt = nullptr;
  int32_t *bc_idx = nullptr;
  double *bc_w = nullptr;
};
