// Launch descriptors shared by the stepping kernels and the host driver.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ib_internal.h"

namespace ib {

// LDS tile of the 3D IB patch (points of support radius <= kTileHalo + 1/2).  Tiles are
// aligned laterally; in depth a tile starts at its first point and spans kTileZ planes, so
// that the thin layer of IB points under the surface falls into few, full tiles.
constexpr int kTileX = 8, kTileY = 8, kTileZ = 16, kTileHalo = 4;
constexpr int kTileMaxPoints = 512;   // longer tile lists are split

struct StepArgs {
  int prec;
  int ndim, M;
  int nx, ny, nz;
  int64_t pitch, vol;
  int nshots;
  int zchunk;
  int variant;          // 3D M=8 interior kernel: 0 basic, 1 pipelined 64x16, 2 pipelined 64x32
  int patch_variant;    // tiled IB patch: bit0 scalar records + weights fetched before staging, bit1 DPP sum
  // per 64 x 16 and 64 x 32 interior tile: the planes [x, y) that hold interior nodes of its
  // columns (3D eighth-order interior kernels)
  const int2 *zrange16, *zrange32;
  int zfirst, zlast;    // planes [zfirst, zlast) hold all interior nodes (generic interior kernel)
  const void *un;       // p^n
  void *um;             // p^{n-1} in (plain form), p^{n+1} out
  void *dd;             // increment form: d^n = p^n - p^{n-1} in, d^{n+1} out (null: plain form)
  const void *K;
  const void *sx, *sy, *sz;
  // IB patch
  int64_t nib;
  const uint32_t *rec;
  const void *pinfo;          // dense-range point records of the tiled points, tile order
  const void *pinfo_tm;       // compact-record point records of the tiled points, tile order
  const void *dense;          // dense-range weights (state precision)
  const int4 *tiles;          // [ntiles + 1]: x0, y0, z0, first point (the last holds the end)
  int ntiles;
  // column-run records of the tiled points (patch variants 8 and 9): entries (state
  // precision), per point (entry offset, packed LDS position) and scale in tile order, first
  // data plane per grid column, column tables
  const void *wcol;
  const uint2 *crec;
  const void *cscale;
  const int16_t *zfcol;
  const int32_t *coltab;
  const void *pinfo_wide;     // points handled by the gather kernel
  int64_t nwide;
  // second stream and events on which the gather kernel of the wide points runs beside
  // the tiled kernel (null: both on the step's stream)
  hipStream_t aux;
  hipEvent_t ev_fork, ev_join;
  // io_merge: the patch launch (the column-run kernel in 3D, the gather kernel in 2D) also
  // injects this step's sources and samples the receivers for the step before (its p^n);
  // the state allows it when no source node is an IB point and no boundary values are set.
  // sample_prev: this step samples the step before.
  int io_merge, sample_prev;
  const int32_t *ball;
  const int32_t *delta;       // linear offsets of the ball lattice points for this layout
  const int32_t *ball_meta;   // [code][2]: start, count
  // sources / receivers
  const int64_t *sidx;
  const void *sw;
  const void *wavelet;
  int64_t wstride;
  int64_t *tcount;      // device [0] next step, [1] step being sampled, [2] first step of the call,
                        // [3] completion count of a patch launch that advances them (io_merge)
  int nrec;
  const int64_t *ridx;
  const void *rw;
  void *traces;
  int64_t nsteps;
  // non-zero boundary values (null: homogeneous conditions): per IB point the scaled
  // contraction F[i][q] of its condition-value weights with g_q, and the time functions
  const int16_t *ib_xyz;
  const void *fF;       // [nib][fnq], state precision
  const void *fs;       // [fnq][fstride], state precision
  int fnq;
  int64_t fstride;
};

void enqueue_step(const StepArgs &a, hipStream_t st);
// receiver sampling alone, of the field u, for the step tcount[1]
void enqueue_sample(const StepArgs &a, const void *u, hipStream_t st);
// whether enqueue_step leaves the sampling of its output to the next step's patch launch
// (io_merge in effect for this state)
bool step_samples_in_patch(const StepArgs &a);
// source injection into u and receiver sampling of u (the sources/receivers fields of a)
void enqueue_source_receivers(const StepArgs &a, void *u, hipStream_t st);

template <typename T>
struct StaggerW {
  T w[kMaxOrder];   // staggered first-derivative weights, offsets -(M-1)/2 .. (M-1)/2
};

// One step of the first-order form (velocity then pressure, with their modified rows).
struct PVArgs {
  int prec, ndim, M, nv;
  int nx, ny, nz;
  int64_t pitch, vol;
  int nshots;
  void *p, *v;                 // p [shot][vol], v [shot][nv][vol]
  const void *kp, *kv;         // dt c^2 / h at interior p nodes; dt / h at interior v nodes [nv][vol]
  const uint8_t *vcls[3];      // classes of the v_n nodes ([z][y][x], bit0 interior): the 3D
  double fv;                   // kernels use (class & 1) * dt / h in place of kv
  const void *sx, *sy, *sz;
  int64_t nrows_g, nrows_d;    // gradient rows (into v), divergence rows (into p)
  const int64_t *g_node, *g_start, *d_node, *d_start;
  const uint32_t *g_enode, *d_enode;   // entry source nodes: padded index + field * vol (< 2^32)
  const void *g_scale, *g_w, *d_scale, *d_w;
  int g_lanes, d_lanes;        // lanes per modified row (8 for short rows, else 16)
  const int2 *zr4;             // 3D: per 64 x 4 column block, the planes [x, y) that hold
                               // interior p or v nodes of its columns
  // io_merge: the rows launches carry the sources and receivers.  The gradient rows of a
  // step sample the receivers for the step before (sample_prev), from p; the divergence
  // rows inject this step's sources into p and advance the step counter.
  int io_merge, sample_prev;
  const int64_t *sidx, *ridx;
  const void *sw, *rw, *wavelet;
  int64_t wstride, nsteps;
  int nrec;
  void *traces;
  int64_t *tcount;
};
void enqueue_pv_step(const PVArgs &a, hipStream_t st);
void enqueue_interior_only(const StepArgs &a, hipStream_t st);
void enqueue_patch_only(const StepArgs &a, hipStream_t st);
size_t pinfo_bytes(int prec);
size_t pinfo_dense_bytes(int prec);
void enqueue_make_pinfo_dense(int prec, const int16_t *xyz, const int32_t *first, const int32_t *count,
                              const uint32_t *doff, const void *scale, const int32_t *perm, int64_t n, void *out,
                              hipStream_t st);

// One adjoint step (lambda^m from lambda^{m+1}, lambda^{m+2}) and its gradient term.
struct AdjArgs {
  int prec, ndim, M;
  int nx, ny, nz;
  int64_t pitch, vol;
  int nshots;
  const void *lam1;      // mu^{m+1} = K lambda^{m+1}
  void *lam2;            // mu^m after the interior stencil (the forward kernel on mu)
  void *lamd;            // increment form: mu^m - mu^{m+1} (null: plain form)
  const void *K, *sx, *sy, *sz;
  // transposed IB rows (receiving nodes, run offsets, IB point and weight per entry)
  int64_t nj;
  const uint32_t *jnode, *joff, *jsrc;
  const void *jD, *jw;   // jD = K_j / (1 + s_j) at the receiving node
  const int16_t *ibxyz;  // IB points (x, y, z, code)
  void *vals;            // scratch [nib][nshots]: mu^{m+1} at the IB points
  int64_t nib;
  // transposed receivers
  int64_t nrn;
  const int64_t *rnode, *roff;
  const int32_t *rrec;
  const void *rD, *rw;   // rD = K_j / (1 + s_j)
  const void *res;       // [nshots][nt][nrec]
  int64_t nt;
  int nrec;
  int64_t step;          // m - 1
  // gradient: gK += mu^m (K L u^{m-1}), K L u^{m-1} recovered from three time levels;
  // dJ/dK = gK / K^2
  double *gK;
  // plain form: u^m, u^{m-1}, u^{m-2}; increment form (u1 null): u2 = d^m, u0 = d^{m-1}
  const void *u2, *u1, *u0;
  const int64_t *sidx;   // source injection of step m - 1 (subtracted from the recovery)
  const void *sw, *wavelet;
  int64_t wstride;
};
void enqueue_adjoint_step(const AdjArgs &a, hipStream_t st);
void enqueue_adj_D(int prec, const uint32_t *jnode, int64_t nj, const void *K, const void *sx, const void *sy,
                   const void *sz, int ny, int64_t pitch, void *D, hipStream_t st);
void enqueue_scale_by_K(int prec, void *v, const int64_t *node, int64_t n, const void *K, hipStream_t st);
ib_status adjoint_table_build(ib_weights *w, hipStream_t st);
void enqueue_grad_out(int prec, const double *gK, const void *K, double *out, int nx, int ny, int nz, int64_t pitch,
                      double dt_over_h, hipStream_t st);
void enqueue_make_pinfo(int prec, const int16_t *xyz, const uint32_t *roff, const void *scale, const int32_t *perm,
                        int64_t n, void *out, hipStream_t st);
void enqueue_make_delta(const int32_t *ball, int n, int64_t pitch, int64_t plane, int32_t *delta, hipStream_t st);

}  // namespace ib
