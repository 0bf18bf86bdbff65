// C ABI: argument checking, ownership, state management and the step driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cfloat>
#include <climits>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ib_internal.h"
#include "step.h"

namespace ib {
ib_status geometry_build(ib_weights *w, const double *height_dev, hipStream_t st);
ib_status ib_points_build(ib_weights *w, hipStream_t st);
ib_status weights_build(ib_weights *w, const int64_t *col_off_dev, hipStream_t st);
ib_status pv_build(ib_weights *w, const int64_t *col_off_dev, hipStream_t st);
ib_status mulder_build(ib_weights *w, hipStream_t st);
const char *last_error_text();
}  // namespace ib

using namespace ib;

// Time checkpoints of one forward run: [count][2][nshots * vol] in the state precision,
// slot 0 = p^{kC}, slot 1 = p^{kC-1} (plain form) or d^{kC} (increment form).
struct ib_checkpoints {
  uint64_t owner = 0;          // uid of the state whose forward run wrote them
  void *data = nullptr;
  size_t bytes = 0;
  int64_t nt = 0, every = 0, count = 0;
};

struct ib_state {
  uint64_t uid = 0;            // unique per state in this process
  const ib_weights *w = nullptr;
  int prec = IB_F32;
  int nshots = 1;
  int64_t pitch = 0, vol = 0;
  size_t esz = 4;
  void *buf[2] = {nullptr, nullptr};
  int cur = 0;                 // buf[cur] holds p^n
  // increment form (FP32 second-order states): dbuf holds d^n = p^n - p^{n-1} and
  // buf[1 - cur] only receives p^{n+1}
  bool incr = false;
  void *dbuf = nullptr;
  void *K = nullptr, *sx = nullptr, *sy = nullptr, *sz = nullptr;
  void *scale = nullptr;
  void *pinfo = nullptr;       // all points, memory order (gradient kernels)
  void *pinfo_t = nullptr;     // tiled points, tile order
  void *pinfo_w = nullptr;     // wide-support points
  void *pinfo_tm = nullptr;    // tiled points, compact records
  uint2 *crec = nullptr;       // tiled points, column-run records: entry offset, packed LDS position
  void *cscale = nullptr;      // tiled points' scales, tile order
  int4 *tiles = nullptr;
  int ntiles = 0;
  int64_t nwide = 0;
  int2 *zrange16 = nullptr, *zrange32 = nullptr;   // interior tiles' plane ranges (3D, M = 8)
  int2 *zr4 = nullptr;         // first-order form, 3D: plane ranges of the 64 x 4 column blocks
  int zfirst = 0, zlast = 0;   // planes [zfirst, zlast) hold every interior node
  hipStream_t aux = nullptr;   // the wide points' gather kernel runs here (3D, both kinds of points)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int32_t *delta = nullptr;
  int64_t *sidx = nullptr;
  void *sw = nullptr;
  int nrec = 0;
  int64_t *ridx = nullptr;
  void *rw = nullptr;
  int64_t *tcount = nullptr;   // device [3]
  int64_t t = 0;
  double dt = 0.0;
  int zchunk = 0;
  int zchunk_auto = 0;
  int variant = 1;
  int patch_variant = 4;
  // sources injected and receivers sampled inside the patch launch (second-order form) or
  // the rows launches (first-order form); no source node is an IB point or a modified row
  bool io_merge = false;
  // captured graphs of two steps and of kLongGraph steps (the same two-step sequence
  // repeated: fewer launches, each of which costs several microseconds of idle device)
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  hipGraph_t graph[2] = {nullptr, nullptr};
  const void *g_wavelet = nullptr;
  void *g_traces = nullptr;
  int64_t g_wstride = 0, g_nsteps = 0;
  int g_cur = 0;
  // first-order form: p in buf[0], velocities [shot][nv][vol], coefficients, modified rows
  int form = 0, nv = 0;
  void *vbuf = nullptr, *kv = nullptr;
  int64_t nrows_g = 0, nrows_d = 0;
  int g_lanes = 16, d_lanes = 16;
  int64_t *g_node = nullptr, *g_start = nullptr, *d_node = nullptr, *d_start = nullptr;
  uint32_t *g_enode = nullptr, *d_enode = nullptr;   // source node (padded index + field offset)
  void *g_scale = nullptr, *g_w = nullptr, *d_scale = nullptr, *d_w = nullptr;
  // host copies needed by the adjoint
  std::vector<double> ax, ay, az;
  std::vector<int64_t> ridx_h;
  std::vector<int64_t> dnode_h;   // first-order form: the divergence rows' p nodes, sorted
  std::vector<double> rw_h;
  // checkpoints written by ib_forward (ib_forward_ckpt writes caller-held ones)
  ib_checkpoints own;
  // watchdog: after every ``watch_every`` steps a scan of p^n (all shots) flags a value that
  // is not finite or exceeds watch_limit in magnitude: wflag[0] = 1, wflag[1] = the least
  // step count at which a scan saw one.  The flags are copied to pinned host memory behind
  // the scan (event ev_watch) and read at the next call, without waiting.
  int64_t watch_every = 100;
  double watch_limit = 1e30;
  int64_t since_watch = 0;
  int32_t *wflag = nullptr;
  int32_t *wflag_h = nullptr;
  hipEvent_t ev_watch = nullptr;
  bool watch_pending = false;
  bool tripped = false;
  int64_t trip_step = -1;
  // adjoint work space and transposed tables (built on first use)
  bool adj_ready = false;
  int64_t nj = 0, nrn = 0;
  int64_t *rnode = nullptr, *roff = nullptr;
  int32_t *rrec = nullptr;
  void *jD = nullptr, *ibvals = nullptr, *rD = nullptr, *rwt = nullptr;
  // non-zero boundary values (ib_state_set_forcing): F [nib][fnq] and the time functions
  // [fnq][flen], state precision; fF == nullptr: homogeneous conditions
  void *fF = nullptr, *fs = nullptr;
  int fnq = 0;
  int64_t flen = 0;
};

// steps in the long captured graph (even: the two-step sequence repeated)
constexpr int64_t kLongGraph = 16;

static void drop_graphs(ib_state *S) {
  for (int k = 0; k < 2; ++k) {
    if (S->gexec[k]) (void)hipGraphExecDestroy(S->gexec[k]);
    if (S->graph[k]) (void)hipGraphDestroy(S->graph[k]);
    S->gexec[k] = nullptr;
    S->graph[k] = nullptr;
  }
}

namespace {

// frees a temporary device buffer on every way out of its scope
template <typename P>
struct FreeOnExit {
  P *&p;
  ~FreeOnExit() {
    dfree(p);
    p = nullptr;
  }
};

void watch_reset(ib_state *S, hipStream_t st);
bool bad(const void *p) { return p == nullptr; }

StepArgs make_args(ib_state *st, const void *wavelet, int64_t wstride, void *traces, int64_t nsteps, int cur) {
  const ib_weights *w = st->w;
  StepArgs a{};
  a.prec = st->prec;
  a.ndim = w->ndim;
  a.M = w->M;
  a.nx = (int)w->nx;
  a.ny = (int)w->ny;
  a.nz = (int)w->nz;
  a.pitch = st->pitch;
  a.vol = st->vol;
  a.nshots = st->nshots;
  a.zchunk = st->zchunk;
  a.variant = st->variant;
  a.patch_variant = st->patch_variant;
  a.un = st->buf[cur];
  a.um = st->buf[1 - cur];
  a.dd = st->incr ? st->dbuf : nullptr;
  a.K = st->K;
  a.sx = st->sx;
  a.sy = st->sy;
  a.sz = st->sz;
  a.nib = w->nib;
  a.rec = (st->prec == IB_F32) ? w->rec32 : w->rec64;
  a.pinfo = st->pinfo_t;
  a.dense = (st->prec == IB_F32) ? (const void *)w->dense32 : (const void *)w->dense64;
  a.tiles = st->tiles;
  a.ntiles = st->ntiles;
  a.pinfo_wide = st->pinfo_w;
  a.pinfo_tm = st->pinfo_tm;
  a.wcol = (st->prec == IB_F32) ? (const void *)w->col32 : (const void *)w->col64;
  a.crec = st->crec;
  a.cscale = st->cscale;
  a.zfcol = w->zfirst;
  a.coltab = w->col_tab;
  a.nwide = st->nwide;
  a.zrange16 = st->zrange16;
  a.zfirst = st->zfirst;
  a.zlast = st->zlast;
  a.zrange32 = st->zrange32;
  a.aux = st->aux;
  a.ev_fork = st->ev_fork;
  a.ev_join = st->ev_join;
  a.delta = st->delta;
  a.ball = w->ball;
  a.ball_meta = w->ball_meta;
  a.sidx = st->sidx;
  a.sw = st->sw;
  a.wavelet = wavelet;
  a.wstride = wstride;
  a.tcount = st->tcount;
  a.io_merge = st->io_merge ? 1 : 0;
  a.sample_prev = 0;
  a.nrec = st->nrec;
  a.ridx = st->ridx;
  a.rw = st->rw;
  a.traces = traces;
  a.nsteps = nsteps;
  a.ib_xyz = w->ib_xyz;
  a.fF = st->fF;
  a.fs = st->fs;
  a.fnq = st->fnq;
  a.fstride = st->flen;
  return a;
}

template <typename T>
__global__ void k_make_K(const double *vel, const uint8_t *cls, T *K, int nx, int ny, int nz, int64_t pitch,
                         double f) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t N = (int64_t)nx * ny * nz;
  if (i >= N) return;
  int x = (int)(i % nx);
  int64_t r = i / nx;
  int y = (int)(r % ny), z = (int)(r / ny);
  double v = vel[i];
  double k = (cls[i] & 1) ? (v * f) * (v * f) : 0.0;
  K[((size_t)z * ny + y) * pitch + x] = (T)k;
}

template <typename T>
__global__ void k_make_coef(const double *vel, const uint8_t *cls, T *K, int nx, int ny, int nz, int64_t pitch,
                            double f, int use_vel) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t N = (int64_t)nx * ny * nz;
  if (i >= N) return;
  int x = (int)(i % nx);
  int64_t r = i / nx;
  int y = (int)(r % ny), z = (int)(r / ny);
  double k = (cls[i] & 1) ? (use_vel ? f * vel[i] * vel[i] : f) : 0.0;
  K[((size_t)z * ny + y) * pitch + x] = (T)k;
}

template <typename T>
__global__ void k_make_scale(const int16_t *xyz, int64_t nib, const double *vel, int nx, int ny, double f,
                             const double *sx, const double *sy, const double *sz, T *scale) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nib) return;
  int x = xyz[i * 4], y = xyz[i * 4 + 1], z = xyz[i * 4 + 2];
  double v = vel[((int64_t)z * ny + y) * nx + x];
  double k = (v * f) * (v * f);
  double s = sx[x] + sy[y] + sz[z];
  scale[i] = (T)(k / (1.0 + s));
}

// p^{n-1} of an increment-form state: dir 0 writes p^n - d^n to the caller's dense
// buffer, dir 1 sets d^n = p^n - (the caller's p^{n-1}) at interior nodes (mask != 0) and 0
// elsewhere
template <typename T>
__global__ void k_field_prev(const T *p, T *d, T *user, const T *mask, int nx, int ny, int nz, int64_t pitch, int dir) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nx * ny * nz) return;
  const int64_t x = i % nx, r = i / nx;
  const size_t c = (size_t)r * pitch + x;
  if (dir == 0)
    user[i] = p[c] - d[c];
  else
    d[c] = (mask[c] != T(0)) ? p[c] - user[i] : T(0);
}

// a field written by the caller keeps zeros at the nodes where the mask is zero (exterior
// nodes: the method takes the wavefield as zero there)
template <typename T>
__global__ void k_mask_field(T *f, const T *mask, int nx, int ny, int nz, int64_t pitch) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nx * ny * nz) return;
  const int64_t x = i % nx, r = i / nx;
  const size_t c = (size_t)r * pitch + x;
  if (mask[c] == T(0)) f[c] = T(0);
}

template <typename T>
__global__ void k_gather_scale(const T *scale, const int32_t *perm, int64_t n, T *out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) out[j] = scale[perm[j]];
}

// step counter of a call: [0] next step, [1] step being sampled, [2] first step
__global__ void k_set_counter(int64_t *tc, int64_t t, int64_t t0) {
  tc[0] = t;
  tc[1] = t;
  tc[2] = t0;
  tc[3] = 0;
}

std::vector<double> damping_axis(int64_t n, int width, double dmax, double dt, bool both) {
  std::vector<double> out(n, 0.0);
  if (width <= 0) return out;
  for (int64_t i = 0; i < n; ++i) {
    double l = 0.0;
    if (both) l = std::max(l, (double)width - (double)i);
    l = std::max(l, (double)i - (double)(n - 1 - width));
    l = std::max(l, 0.0);
    double d = dmax * (l / width) * (l / width);
    out[i] = d * dt / 2.0;
  }
  return out;
}

// multilinear corners of a point (grid units); -1 where the weight is exactly zero
bool corners(const ib_weights *w, const double *pos_m, int64_t idx[8], double wt[8], int64_t pitch,
             bool padded) {
  double g[3] = {pos_m[0] / w->h, 0.0, 0.0};
  if (w->ndim == 3) {
    g[1] = pos_m[1] / w->h;
    g[2] = pos_m[2] / w->h;
  } else {
    g[2] = pos_m[1] / w->h;
  }
  int b[3];
  double f[3];
  for (int n = 0; n < 3; ++n) {
    b[n] = (int)floor(g[n]);
    f[n] = g[n] - b[n];
  }
  for (int c = 0; c < 8; ++c) {
    idx[c] = -1;
    wt[c] = 0.0;
  }
  int ncorner = (w->ndim == 3) ? 8 : 4;
  for (int c = 0; c < ncorner; ++c) {
    int bx = c & 1, by = 0, bz;
    if (w->ndim == 3) {
      by = (c >> 1) & 1;
      bz = (c >> 2) & 1;
    } else {
      bz = (c >> 1) & 1;
    }
    double wx = bx ? f[0] : 1.0 - f[0];
    double wy = (w->ndim == 3) ? (by ? f[1] : 1.0 - f[1]) : 1.0;
    double wz = bz ? f[2] : 1.0 - f[2];
    double ww = wx * wy * wz;
    if (ww == 0.0) continue;
    int64_t x = ((b[0] + bx) % w->nx + w->nx) % w->nx;
    int64_t y = (w->ndim == 3) ? ((b[1] + by) % w->ny + w->ny) % w->ny : 0;
    int64_t z = b[2] + bz;
    if (z < 0 || z >= w->nz) return false;
    idx[c] = padded ? (z * w->ny + y) * pitch + x : (z * w->ny + y) * w->nx + x;
    wt[c] = ww;
  }
  return true;
}

// Tile-depth autotuner of the 3D eighth-order interior kernel: times each candidate
// (HIP events, on the state's own buffers, whose contents it leaves unchanged because
// they are zero) and keeps the fastest.
ib_status autotune_interior(ib_state *S, hipStream_t st) {
  const ib_weights *w = S->w;
  if (!(w->ndim == 3 && w->M == 8)) return IB_OK;
  std::vector<int> cands;
  for (int d : {2, 3, 4, 5, 6, 8, 10, 12, 14, 16, 20, 24}) {
    int zc = (int)((w->nz + d - 1) / d);
    if (zc >= 12 && std::find(cands.begin(), cands.end(), zc) == cands.end()) cands.push_back(zc);
  }
  hipEvent_t e0, e1;
  IB_HIP(hipEventCreate(&e0));
  IB_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int bestzc = S->zchunk;
  int bestv = 1;
  // two passes over every (variant, zchunk) pair, each timed over 8 launches after 2
  // warm-up launches; the minimum of the two passes is kept (clocks ramp up during the first)
  const int variants[3] = {1, 3, 4};
  const int nv = 3;
  std::vector<float> tbest(nv * cands.size(), 1e30f);
  for (int pass = 0; pass < 2; ++pass)
    for (int cand = 0; cand < nv * (int)cands.size(); ++cand) {
      S->variant = variants[cand % nv];
      S->zchunk = cands[cand / nv];
      StepArgs a = make_args(S, nullptr, 0, nullptr, 0, S->cur);
      for (int i = 0; i < 2; ++i) enqueue_interior_only(a, st);
      IB_HIP(hipEventRecord(e0, st));
      for (int i = 0; i < 8; ++i) enqueue_interior_only(a, st);
      IB_HIP(hipEventRecord(e1, st));
      IB_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      IB_HIP(hipEventElapsedTime(&ms, e0, e1));
      tbest[cand] = std::min(tbest[cand], ms);
    }
  for (int cand = 0; cand < nv * (int)cands.size(); ++cand)
    if (tbest[cand] < best) {
      best = tbest[cand];
      bestzc = cands[cand / nv];
      bestv = variants[cand % nv];
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  S->variant = bestv;
  S->zchunk = bestzc;
  S->zchunk_auto = bestzc;
  return IB_OK;
}

}  // namespace

namespace {
// a(x_b): periodic bilinear (lat == 1: linear) interpolation of the per-column samples
__global__ void k_bp_robin(double *bp, int64_t nb, const double *a, int nx, int ny, int lat) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nb) return;
  double *o = bp + j * 8;
  const double x = o[3], y = (lat == 2) ? o[4] : 0.0;
  const double fx0 = floor(x), fy0 = floor(y);
  const double tx = x - fx0, ty = y - fy0;
  auto wrap = [](long long i, int n) { return (int)(((i % n) + n) % n); };
  const int i0 = wrap((long long)fx0, nx), i1 = wrap((long long)fx0 + 1, nx);
  double v;
  if (lat == 1) {
    v = (1.0 - tx) * a[i0] + tx * a[i1];
  } else {
    const int j0 = wrap((long long)fy0, ny), j1 = wrap((long long)fy0 + 1, ny);
    v = (1.0 - tx) * (1.0 - ty) * a[(int64_t)j0 * nx + i0] + tx * (1.0 - ty) * a[(int64_t)j0 * nx + i1] +
        (1.0 - tx) * ty * a[(int64_t)j1 * nx + i0] + tx * ty * a[(int64_t)j1 * nx + i1];
  }
  o[6] = v;
}
}  // namespace

namespace {
struct HPow {
  double v[8];
};

// F[i][q] = scale_i h^{o_q} sum over the point's entries of condition q of weight * g[b][q]
template <typename T>
__global__ void k_forcing_setup(int64_t nib, const int64_t *off, const int32_t *cnt, const int32_t *idx,
                                const double *wv, const double *g, int nq, HPow hp, const T *scale, T *F) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nib) return;
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int64_t e0 = off[i], e1 = off[i] + cnt[i];
  for (int64_t e = e0; e < e1; ++e) {
    const int v = idx[e];
    const int b = v >> 3, q = v & 7;
    if (q < nq) acc[q] += wv[e] * g[(int64_t)b * nq + q];
  }
  const double sc = (double)scale[i];
  for (int q = 0; q < nq; ++q) F[i * nq + q] = (T)(sc * hp.v[q] * acc[q]);
}
}  // namespace

extern "C" {

int32_t ib_abi_version(void) { return IB_ABI_VERSION; }

const char *ib_last_error(void) { return ib::last_error_text(); }

ib_status ib_build_weights(const ib_grid *g, const double *height_dev, const ib_params *p, void *stream,
                           ib_weights **out) {
  auto t0 = std::chrono::steady_clock::now();
  if (!g || !p || !out || bad(height_dev)) {
    set_error("ib_build_weights: null argument");
    return IB_ERR_ARG;
  }
  *out = nullptr;
  if (g->ndim != 2 && g->ndim != 3) {
    set_error("ndim must be 2 or 3 (got %d)", g->ndim);
    return IB_ERR_ARG;
  }
  if (p->form != IB_FORM_P2 && p->form != IB_FORM_PV1) {
    set_error("unsupported form %d", p->form);
    return IB_ERR_ARG;
  }
  if (p->form == IB_FORM_PV1 && g->ndim == 3 && p->space_order >= 2 && p->space_order <= kMaxOrder &&
      3 * n_terms(p->space_order, 3) > 192) {
    // the divergence family couples the three velocity blocks of the Taylor basis
    set_error("the 3D first-order form needs space_order <= 4 (its coupled velocity system has %d unknowns, "
              "the solver takes 192)", 3 * n_terms(p->space_order, 3));
    return IB_ERR_ARG;
  }
  if (p->method != IB_METHOD_ND && p->method != IB_METHOD_1D) {
    set_error("unsupported method %d", p->method);
    return IB_ERR_ARG;
  }
  if (p->keep_bc_weights != 0 && p->keep_bc_weights != 1) {
    set_error("keep_bc_weights must be 0 or 1 (got %d)", p->keep_bc_weights);
    return IB_ERR_ARG;
  }
  if (p->keep_bc_weights && (p->form != IB_FORM_P2 || p->method != IB_METHOD_ND)) {
    set_error("condition-value weights are kept for the second-order form with the N-D method only");
    return IB_ERR_ARG;
  }
  if (p->method == IB_METHOD_1D && (p->form != IB_FORM_P2 || p->surface != IB_SURF_FREE)) {
    // the reduction to 1D is given for the free-surface conditions of the pressure form
    set_error("the 1D extrapolation method is defined for the second-order form with a free surface");
    return IB_ERR_ARG;
  }
  if (p->form == IB_FORM_PV1 && p->surface != IB_SURF_FREE) {
    // the method's first-order form is given for the free surface (zero pressure and the
    // divergence hierarchy); a rigid-surface velocity row set is not part of it
    set_error("the first-order form supports the free surface only");
    return IB_ERR_ARG;
  }
  if (p->form == IB_FORM_PV1 && !(p->eta_v >= 0.0 && p->eta_v <= 1.0)) {
    set_error("eta_v must be in [0, 1] (got %g)", p->eta_v);
    return IB_ERR_ARG;
  }
  if (p->surface != IB_SURF_FREE && p->surface != IB_SURF_RIGID && p->surface != IB_SURF_ROBIN) {
    set_error("unsupported surface %d", p->surface);
    return IB_ERR_ARG;
  }
  if ((p->surface == IB_SURF_ROBIN) != (p->robin_dev != nullptr)) {
    set_error("robin_dev is required by the mixed (robin) surface and only by it");
    return IB_ERR_ARG;
  }
  if (p->surface == IB_SURF_ROBIN && (p->form != IB_FORM_P2 || p->method != IB_METHOD_ND)) {
    set_error("the mixed (robin) surface is built for the second-order form with the N-D method");
    return IB_ERR_ARG;
  }
  if (p->space_order < 2 || p->space_order > kMaxOrder || (p->space_order & 1)) {
    set_error("space_order must be even in [2, %d] (got %d)", kMaxOrder, p->space_order);
    return IB_ERR_ARG;
  }
  if (p->max_radius_steps < 0 || p->space_order + 1 + 2 * p->max_radius_steps + 2 > kMaxRadiusCode) {
    set_error("max_radius_steps out of range (%d)", p->max_radius_steps);
    return IB_ERR_ARG;
  }
  if (p->min_basis_order < 1 || p->min_basis_order > p->space_order) {
    set_error("min_basis_order must be in [1, space_order] (got %d)", p->min_basis_order);
    return IB_ERR_ARG;
  }
  if (!(p->eta >= 0.0 && p->eta <= 1.0)) {
    set_error("eta must be in [0, 1] (got %g)", p->eta);
    return IB_ERR_ARG;
  }
  if (!(g->h > 0.0)) {
    set_error("grid increment must be positive");
    return IB_ERR_ARG;
  }
  {
    // the IB patch kernel holds a support ball's mask in one wavefront (<= 2048 points)
    BallTables bt;
    int maxc = p->space_order + 1 + 2 * p->max_radius_steps;
    bt.build(g->ndim, maxc);
    if (bt.count[maxc] > 2048) {
      set_error("largest support ball (radius %.1f) exceeds 2048 lattice points; lower max_radius_steps", maxc / 2.0);
      return IB_ERR_ARG;
    }
  }
  ib_weights *w = new ib_weights();
  w->ndim = g->ndim;
  w->nx = g->n[0];
  w->ny = (g->ndim == 3) ? g->n[1] : 1;
  w->nz = g->n[g->ndim - 1];
  w->N = w->nx * w->ny * w->nz;
  w->h = g->h;
  w->prm = *p;
  w->M = p->space_order;
  w->pitch = (w->nx + 31) / 32 * 32;
  if (w->nx < 16 || w->nz < 16 || (g->ndim == 3 && w->ny < 16) || w->nx > 32000 || w->ny > 32000 ||
      w->nz > 32000 || w->N >= (int64_t)1 << 31) {
    set_error("grid extents must be in [16, 32000] with fewer than 2^31 nodes");
    delete w;
    return IB_ERR_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  int64_t *col_off = nullptr;   // solver column offsets, released by the body or below
  // every failure in the body returns through here, which frees the partly built table
  auto build = [&]() -> ib_status {
    IB_HIP(hipGetDevice(&w->device));
    ib_status s = geometry_build(w, height_dev, st);
    if (s != IB_OK) {
      return s;
    }
    if (p->surface == IB_SURF_ROBIN && w->nb > 0) {
      // the coefficient at each boundary point, kept in slot 6 of its record
      hipLaunchKernelGGL(k_bp_robin, dim3((unsigned)((w->nb + 255) / 256)), dim3(256), 0, st, w->bp, w->nb,
                         p->robin_dev, (int)w->nx, (int)w->ny, w->ndim - 1);
      IB_HIP(hipGetLastError());
      IB_HIP(hipStreamSynchronize(st));
    }
    w->prm.robin_dev = nullptr;   // borrowed for this call only
    // the surface band must stay clear of the top and bottom of the box
    {
      std::vector<double> hs(w->nx * w->ny);
      IB_HIP(hipMemcpy(hs.data(), w->Hs, hs.size() * 8, hipMemcpyDeviceToHost));
      double lo = *std::min_element(hs.begin(), hs.end()), hi = *std::max_element(hs.begin(), hs.end());
      double margin = (w->M + 1 + 2 * p->max_radius_steps) / 2.0 + w->M / 2 + 2;
      if (lo < margin || hi > (double)(w->nz - 1) - margin) {
        set_error("surface depth range [%.2f, %.2f] cells must keep %.1f cells from the top and bottom", lo, hi, margin);
        return IB_ERR_ARG;
      }
    }
    w->form = p->form;
    if (w->form == IB_FORM_P2 && (s = ib_points_build(w, st)) != IB_OK) {
      return s;
    }
    // boundary points are stored per column: rebuild column offsets for the solver
    {
      int64_t ncol = w->nx * w->ny;
      std::vector<double> bp(w->nb * 8);
      if (w->nb) IB_HIP(hipMemcpy(bp.data(), w->bp, bp.size() * 8, hipMemcpyDeviceToHost));
      std::vector<int64_t> off(ncol + 1, 0);
      for (int64_t j = 0; j < w->nb; ++j) {
        int64_t c = (int64_t)bp[j * 8 + 1] * w->nx + (int64_t)bp[j * 8 + 0];
        off[c + 1]++;
      }
      for (int64_t c = 0; c < ncol; ++c) off[c + 1] += off[c];
      if ((s = dalloc_t(&col_off, ncol + 1)) != IB_OK) {
        return s;
      }
      IB_HIP(hipMemcpy(col_off, off.data(), (ncol + 1) * 8, hipMemcpyHostToDevice));
    }
    if (w->form == IB_FORM_PV1)
      s = pv_build(w, col_off, st);
    else
      s = (p->method == IB_METHOD_1D) ? mulder_build(w, st) : weights_build(w, col_off, st);
    dfree(col_off);
    col_off = nullptr;
    if (s != IB_OK) {
      return s;
    }
    // statistics
    {
      std::vector<uint8_t> cls(w->N);
      IB_HIP(hipMemcpy(cls.data(), w->node_class, w->N, hipMemcpyDeviceToHost));
      int64_t ni = 0;
      for (auto c : cls) ni += (c & 1);
      w->stats.n_nodes = w->N;
      w->stats.n_interior = ni;
      w->stats.n_boundary_points = w->nb;
      w->stats.n_ib = w->nib;
    }
    IB_HIP(hipStreamSynchronize(st));
    w->stats.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return IB_OK;
  };
  const ib_status status = build();
  if (status != IB_OK) {
    dfree(col_off);
    ib_weights_free(w);
    return status;
  }
  *out = w;
  return IB_OK;
}

ib_status ib_weights_stats(const ib_weights *w, ib_stats *out) {
  if (!w || !out) {
    set_error("ib_weights_stats: null argument");
    return IB_ERR_ARG;
  }
  *out = w->stats;
  return IB_OK;
}

void ib_weights_free(ib_weights *w) {
  if (!w) return;
  dfree(w->Hs);
  dfree(w->node_class);
  dfree(w->bp);
  dfree(w->bp_normal);
  dfree(w->ib_node);
  dfree(w->ib_xyz);
  dfree(w->ib_meta);
  dfree(w->ib_sigma);
  dfree(w->w64);
  dfree(w->rec32);
  dfree(w->rec64);
  dfree(w->rec_off32);
  dfree(w->rec_off64);
  dfree(w->ball);
  dfree(w->ball_meta);
  dfree(w->dense32);
  dfree(w->dense64);
  dfree(w->dense_first);
  dfree(w->dense_count);
  dfree(w->dense_off);
  dfree(w->zfirst), dfree(w->col_tab), dfree(w->col_off), dfree(w->col_cnt), dfree(w->col32), dfree(w->col64);
  for (int n = 0; n < 3; ++n) dfree(w->vcls[n]);
  dfree(w->adj_jnode), dfree(w->adj_joff), dfree(w->adj_jsrc), dfree(w->adj_jw32), dfree(w->adj_jw64);
  dfree(w->bc_off), dfree(w->bc_cnt), dfree(w->bc_idx), dfree(w->bc_w);
  delete w;
}

ib_status ib_weights_copy(const ib_weights *w, int32_t field, void *dst, int64_t bytes) {
  if (!w || !dst) {
    set_error("ib_weights_copy: null argument");
    return IB_ERR_ARG;
  }
  const void *src = nullptr;
  int64_t need = 0;
  switch (field) {
    case IB_FIELD_NODE_CLASS: src = w->node_class; need = w->N; break;
    case IB_FIELD_IB_NODES: src = w->ib_node; need = w->nib * 8; break;
    case IB_FIELD_IB_META: src = w->ib_meta; need = w->nib * 16; break;
    case IB_FIELD_WEIGHTS_F64: src = w->w64; need = w->sumw * 8; break;
    case IB_FIELD_SIGMA: src = w->ib_sigma; need = w->nib * 8; break;
    case IB_FIELD_PV_ROWS:
    case IB_FIELD_PV_ENTRIES:
    case IB_FIELD_VCLASS: {
      if (w->form != IB_FORM_PV1) {
        set_error("ib_weights_copy: field %d exists for the first-order form only", field);
        return IB_ERR_STATE;
      }
      const int64_t nr = (int64_t)w->pv_row_fam.size(), ne = (int64_t)w->pv_ent_w.size();
      need = (field == IB_FIELD_PV_ROWS) ? nr * 24 : (field == IB_FIELD_PV_ENTRIES ? ne * 24 : w->ndim * w->N);
      if (bytes < need) {
        set_error("ib_weights_copy: destination too small (%lld < %lld)", (long long)bytes, (long long)need);
        return IB_ERR_ARG;
      }
      if (field == IB_FIELD_PV_ROWS) {
        int64_t *o = (int64_t *)dst;
        for (int64_t r = 0; r < nr; ++r) {
          o[r * 3] = w->pv_row_fam[r];
          o[r * 3 + 1] = w->pv_row_node[r];
          o[r * 3 + 2] = w->pv_row_start[r + 1] - w->pv_row_start[r];
        }
      } else if (field == IB_FIELD_PV_ENTRIES) {
        double *o = (double *)dst;
        for (int64_t e = 0; e < ne; ++e) {
          o[e * 3] = w->pv_ent_field[e];
          o[e * 3 + 1] = (double)w->pv_ent_node[e];
          o[e * 3 + 2] = w->pv_ent_w[e];
        }
      } else {
        for (int n = 0; n < w->ndim; ++n)
          IB_HIP(hipMemcpy((uint8_t *)dst + n * w->N, w->vcls[n], w->N, hipMemcpyDeviceToHost));
      }
      return IB_OK;
    }
    case IB_FIELD_BC_COUNTS:
    case IB_FIELD_BC_ENTRIES: {
      if (!w->bc_off) {
        set_error("ib_weights_copy: the table was built without condition-value weights (keep_bc_weights = 0)");
        return IB_ERR_STATE;
      }
      std::vector<int64_t> off(w->nib);
      std::vector<int32_t> cnt(w->nib);
      if (w->nib) {
        IB_HIP(hipMemcpy(off.data(), w->bc_off, w->nib * 8, hipMemcpyDeviceToHost));
        IB_HIP(hipMemcpy(cnt.data(), w->bc_cnt, w->nib * 4, hipMemcpyDeviceToHost));
      }
      need = (field == IB_FIELD_BC_COUNTS) ? w->nib * 4 : w->nbc * 24;
      if (bytes < need) {
        set_error("ib_weights_copy: destination too small (%lld < %lld)", (long long)bytes, (long long)need);
        return IB_ERR_ARG;
      }
      if (field == IB_FIELD_BC_COUNTS) {
        std::memcpy(dst, cnt.data(), w->nib * 4);
        return IB_OK;
      }
      std::vector<int32_t> idx(w->nbc);
      std::vector<double> wv(w->nbc);
      if (w->nbc) {
        IB_HIP(hipMemcpy(idx.data(), w->bc_idx, w->nbc * 4, hipMemcpyDeviceToHost));
        IB_HIP(hipMemcpy(wv.data(), w->bc_w, w->nbc * 8, hipMemcpyDeviceToHost));
      }
      double *o = (double *)dst;
      int64_t k = 0;
      for (int64_t i = 0; i < w->nib; ++i)
        for (int64_t e = off[i]; e < off[i] + cnt[i]; ++e, ++k) {
          o[k * 3] = (double)(idx[e] >> 3);
          o[k * 3 + 1] = (double)(idx[e] & 7);
          o[k * 3 + 2] = wv[e];
        }
      return IB_OK;
    }
    case IB_FIELD_BPOINTS: {
      need = w->nb * 7 * 8;
      if (bytes < need) {
        set_error("ib_weights_copy: destination too small (%lld < %lld)", (long long)bytes, (long long)need);
        return IB_ERR_ARG;
      }
      std::vector<double> bp(w->nb * 8);
      if (w->nb) IB_HIP(hipMemcpy(bp.data(), w->bp, bp.size() * 8, hipMemcpyDeviceToHost));
      double *o = (double *)dst;
      for (int64_t j = 0; j < w->nb; ++j) {
        for (int q = 0; q < 7; ++q) o[j * 7 + q] = bp[j * 8 + q];
      }
      return IB_OK;
    }
    default:
      set_error("ib_weights_copy: unknown field %d", field);
      return IB_ERR_ARG;
  }
  if (bytes < need) {
    set_error("ib_weights_copy: destination too small (%lld < %lld)", (long long)bytes, (long long)need);
    return IB_ERR_ARG;
  }
  if (need) IB_HIP(hipMemcpy(dst, src, need, hipMemcpyDeviceToHost));
  return IB_OK;
}

ib_status ib_state_create(const ib_weights *w, const double *vel_dev, double dt, int32_t damp_width, double damp_R,
                          int32_t prec, int32_t nshots, const double *src_pos, int32_t nrec, const double *rec_pos,
                          void *stream, ib_state **out) {
  if (!w || !out || bad(vel_dev) || (nshots > 0 && !src_pos) || (nrec > 0 && !rec_pos)) {
    set_error("ib_state_create: null argument");
    return IB_ERR_ARG;
  }
  *out = nullptr;
  if (prec != IB_F32 && prec != IB_F64) {
    set_error("precision must be IB_F32 or IB_F64");
    return IB_ERR_ARG;
  }
  if (nshots < 1 || nrec < 0 || !(dt > 0.0) || damp_width < 0 || (damp_width > 0 && !(damp_R > 0.0 && damp_R < 1.0))) {
    set_error("ib_state_create: invalid nshots/nrec/dt/damping");
    return IB_ERR_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  ib_state *S = new ib_state();
  static std::atomic<uint64_t> next_uid{1};
  S->uid = next_uid++;
  S->w = w;
  S->prec = prec;
  S->nshots = nshots;
  S->esz = (prec == IB_F32) ? 4 : 8;
  S->pitch = w->pitch;
  S->vol = S->pitch * w->ny * w->nz;
  S->dt = dt;
  S->nrec = nrec;
  S->zchunk = 0;
  // every failure in the body returns through here, which frees the partly built state
  auto build = [&]() -> ib_status {
    ib_status s;
    auto fail = [](ib_status e) { return e; };
    const size_t fbytes = (size_t)S->vol * nshots * S->esz;
    if ((s = dalloc(&S->buf[0], fbytes)) || (s = dalloc(&S->buf[1], fbytes)) || (s = dalloc(&S->K, S->vol * S->esz)))
      return fail(s);
    IB_HIP(hipMemsetAsync(S->buf[0], 0, fbytes, st));
    IB_HIP(hipMemsetAsync(S->buf[1], 0, fbytes, st));
    S->incr = (prec == IB_F32 && w->form == IB_FORM_P2);
    if (S->incr) {
      if ((s = dalloc(&S->dbuf, fbytes))) return fail(s);
      IB_HIP(hipMemsetAsync(S->dbuf, 0, fbytes, st));
    }
    IB_HIP(hipMemsetAsync(S->K, 0, S->vol * S->esz, st));
    const double f = dt / w->h;
    const int T = 256;
    if (prec == IB_F32)
      hipLaunchKernelGGL(k_make_K<float>, dim3((w->N + T - 1) / T), dim3(T), 0, st, vel_dev, w->node_class,
                         (float *)S->K, (int)w->nx, (int)w->ny, (int)w->nz, S->pitch, f);
    else
      hipLaunchKernelGGL(k_make_K<double>, dim3((w->N + T - 1) / T), dim3(T), 0, st, vel_dev, w->node_class,
                         (double *)S->K, (int)w->nx, (int)w->ny, (int)w->nz, S->pitch, f);
    IB_HIP(hipGetLastError());
    // damping tables
    double vmax = 0.0;
    {
      std::vector<double> v(w->N);
      IB_HIP(hipMemcpyAsync(v.data(), vel_dev, w->N * 8, hipMemcpyDeviceToHost, st));
      IB_HIP(hipStreamSynchronize(st));
      for (double x : v) vmax = std::max(vmax, x);
    }
    // d = d_max (l / W)^2: a wave crossing the layer, reflected at its outer edge and
    // crossing back keeps the amplitude fraction R (WKB); the second-order form's damping
    // term attenuates at the rate d / 2, the first-order form's terms at the rate d
    double dmax = (damp_width > 0) ? 3.0 * vmax * std::log(1.0 / damp_R) / (damp_width * w->h) : 0.0;
    if (w->form == IB_FORM_PV1) dmax *= 0.5;
    std::vector<double> ax = damping_axis(w->nx, damp_width, dmax, dt, true);
    std::vector<double> ay = (w->ndim == 3) ? damping_axis(w->ny, damp_width, dmax, dt, true) : std::vector<double>(1, 0.0);
    std::vector<double> az = damping_axis(w->nz, damp_width, dmax, dt, false);
    double *d_ax = nullptr, *d_ay = nullptr, *d_az = nullptr;
    FreeOnExit<double> free_ax{d_ax}, free_ay{d_ay}, free_az{d_az};
    if ((s = dalloc_t(&d_ax, ax.size())) || (s = dalloc_t(&d_ay, ay.size())) || (s = dalloc_t(&d_az, az.size())))
      return fail(s);
    IB_HIP(hipMemcpy(d_ax, ax.data(), ax.size() * 8, hipMemcpyHostToDevice));
    IB_HIP(hipMemcpy(d_ay, ay.data(), ay.size() * 8, hipMemcpyHostToDevice));
    IB_HIP(hipMemcpy(d_az, az.data(), az.size() * 8, hipMemcpyHostToDevice));
    auto upload_cast = [&](const std::vector<double> &v, void **dst) -> ib_status {
      ib_status e = dalloc(dst, v.size() * S->esz);
      if (e) return e;
      if (prec == IB_F32) {
        std::vector<float> t(v.begin(), v.end());
        IB_HIP(hipMemcpy(*dst, t.data(), t.size() * 4, hipMemcpyHostToDevice));
      } else {
        IB_HIP(hipMemcpy(*dst, v.data(), v.size() * 8, hipMemcpyHostToDevice));
      }
      return IB_OK;
    };
    if ((s = upload_cast(ax, &S->sx)) || (s = upload_cast(ay, &S->sy)) || (s = upload_cast(az, &S->sz))) return fail(s);
    S->ax = ax;
    S->ay = ay;
    S->az = az;
    S->form = w->form;
    if (w->form == IB_FORM_PV1) {
      // first-order form: K holds dt c^2 / h at interior p nodes, kv dt / h at interior v nodes
      S->nv = w->ndim;
      if ((int64_t)S->vol * S->nv >= ((int64_t)1 << 32)) {
        // modified-row entries address the velocity fields with 32-bit indices
        set_error("the first-order form needs ndim * padded grid < 2^32 nodes");
        return fail(IB_ERR_ARG);
      }
      const size_t vbytes = (size_t)S->vol * S->nv * nshots * S->esz;
      if ((s = dalloc(&S->vbuf, vbytes)) || (s = dalloc(&S->kv, (size_t)S->vol * S->nv * S->esz))) return fail(s);
      IB_HIP(hipMemsetAsync(S->vbuf, 0, vbytes, st));
      IB_HIP(hipMemsetAsync(S->kv, 0, (size_t)S->vol * S->nv * S->esz, st));
      for (int n = 0; n < S->nv; ++n) {
        char *dst = (char *)S->kv + (size_t)n * S->vol * S->esz;
        if (prec == IB_F32)
          hipLaunchKernelGGL(k_make_coef<float>, dim3((w->N + T - 1) / T), dim3(T), 0, st, vel_dev, w->vcls[n],
                             (float *)dst, (int)w->nx, (int)w->ny, (int)w->nz, S->pitch, f, 0);
        else
          hipLaunchKernelGGL(k_make_coef<double>, dim3((w->N + T - 1) / T), dim3(T), 0, st, vel_dev, w->vcls[n],
                             (double *)dst, (int)w->nx, (int)w->ny, (int)w->nz, S->pitch, f, 0);
      }
      if (prec == IB_F32)
        hipLaunchKernelGGL(k_make_coef<float>, dim3((w->N + T - 1) / T), dim3(T), 0, st, vel_dev, w->node_class,
                           (float *)S->K, (int)w->nx, (int)w->ny, (int)w->nz, S->pitch, dt / w->h, 1);
      else
        hipLaunchKernelGGL(k_make_coef<double>, dim3((w->N + T - 1) / T), dim3(T), 0, st, vel_dev, w->node_class,
                           (double *)S->K, (int)w->nx, (int)w->ny, (int)w->nz, S->pitch, dt / w->h, 1);
      IB_HIP(hipGetLastError());
      // modified rows with their scales, in the state layout
      std::vector<double> velh(w->N);
      IB_HIP(hipMemcpy(velh.data(), vel_dev, w->N * 8, hipMemcpyDeviceToHost));
      auto padded = [&](int64_t node) {
        const int64_t x = node % w->nx, y = (node / w->nx) % w->ny, z = node / (w->nx * w->ny);
        return (z * w->ny + y) * S->pitch + x;
      };
      auto sig = [&](int64_t node) {
        const int64_t x = node % w->nx, y = (node / w->nx) % w->ny, z = node / (w->nx * w->ny);
        return ax[x] + ay[w->ndim == 3 ? y : 0] + az[z];
      };
      std::vector<int64_t> gn, gs(1, 0), ge, dn, ds(1, 0), de;
      std::vector<double> gsc, gw, dsc, dw;
      const int64_t nr = (int64_t)w->pv_row_fam.size();
      for (int64_t r = 0; r < nr; ++r) {
        const int fam = w->pv_row_fam[r];
        const int64_t node = w->pv_row_node[r];
        const bool grad = fam < S->nv;
        for (int64_t e = w->pv_row_start[r]; e < w->pv_row_start[r + 1]; ++e) {
          const int fld = w->pv_ent_field[e];
          const int64_t q = padded(w->pv_ent_node[e]) + (fld >= 0 ? (int64_t)fld * S->vol : 0);
          (grad ? ge : de).push_back(q);
          (grad ? gw : dw).push_back(w->pv_ent_w[e]);
        }
        if (grad) {
          gn.push_back((int64_t)fam * S->vol + padded(node));
          gsc.push_back(f / (1.0 + sig(node)));
          gs.push_back((int64_t)ge.size());
        } else {
          const double c = velh[node];
          dn.push_back(padded(node));
          dsc.push_back((dt * c * c / w->h) / (1.0 + sig(node)));
          ds.push_back((int64_t)de.size());
        }
      }
      S->nrows_g = (int64_t)gn.size();
      S->nrows_d = (int64_t)dn.size();
      S->dnode_h = dn;
      std::sort(S->dnode_h.begin(), S->dnode_h.end());
      // rows of fewer than 40 entries on average take 8 lanes each (more rows per wavefront)
      S->g_lanes = (gn.empty() || ge.size() >= 40 * gn.size()) ? 16 : 8;
      S->d_lanes = (dn.empty() || de.size() >= 40 * dn.size()) ? 16 : 8;
      auto up64 = [&](const std::vector<int64_t> &v, int64_t **d) -> ib_status {
        ib_status e = dalloc_t(d, std::max<size_t>(v.size(), 1));
        if (e) return e;
        if (!v.empty()) IB_HIP(hipMemcpy(*d, v.data(), v.size() * 8, hipMemcpyHostToDevice));
        return IB_OK;
      };
      auto up32 = [&](const std::vector<int64_t> &v, uint32_t **d) -> ib_status {
        std::vector<uint32_t> n32(v.begin(), v.end());
        ib_status e = dalloc_t(d, std::max<size_t>(n32.size(), 1));
        if (e) return e;
        if (!n32.empty()) IB_HIP(hipMemcpy(*d, n32.data(), n32.size() * 4, hipMemcpyHostToDevice));
        return IB_OK;
      };
      if ((s = up64(gn, &S->g_node)) || (s = up64(gs, &S->g_start)) || (s = up32(ge, &S->g_enode)) ||
          (s = up64(dn, &S->d_node)) || (s = up64(ds, &S->d_start)) || (s = up32(de, &S->d_enode)) ||
          (s = upload_cast(gsc.empty() ? std::vector<double>(1, 0.0) : gsc, &S->g_scale)) ||
          (s = upload_cast(gw.empty() ? std::vector<double>(1, 0.0) : gw, &S->g_w)) ||
          (s = upload_cast(dsc.empty() ? std::vector<double>(1, 0.0) : dsc, &S->d_scale)) ||
          (s = upload_cast(dw.empty() ? std::vector<double>(1, 0.0) : dw, &S->d_w)))
        return fail(s);
    } else {
      if ((s = dalloc(&S->scale, std::max<int64_t>(w->nib, 1) * S->esz))) return fail(s);
      if (w->nib > 0) {
        if (prec == IB_F32)
          hipLaunchKernelGGL(k_make_scale<float>, dim3((w->nib + T - 1) / T), dim3(T), 0, st, w->ib_xyz, w->nib, vel_dev,
                             (int)w->nx, (int)w->ny, f, d_ax, d_ay, d_az, (float *)S->scale);
        else
          hipLaunchKernelGGL(k_make_scale<double>, dim3((w->nib + T - 1) / T), dim3(T), 0, st, w->ib_xyz, w->nib,
                             vel_dev, (int)w->nx, (int)w->ny, f, d_ax, d_ay, d_az, (double *)S->scale);
        IB_HIP(hipGetLastError());
      }
      if ((s = dalloc(&S->pinfo, std::max<int64_t>(w->nib, 1) * pinfo_bytes(prec))) ||
          (s = dalloc_t(&S->delta, std::max<size_t>(w->balls.packed.size(), 1))))
        return fail(s);
      enqueue_make_pinfo(prec, w->ib_xyz, prec == IB_F32 ? w->rec_off32 : w->rec_off64, S->scale, nullptr, w->nib,
                         S->pinfo, st);
      {
        // bucket the IB points into LDS tiles (3D); wider supports go to the gather kernel
        std::vector<int16_t> xyz(w->nib * 4);
        if (w->nib) IB_HIP(hipMemcpy(xyz.data(), w->ib_xyz, w->nib * 8, hipMemcpyDeviceToHost));
        std::vector<int32_t> tiled, wide;
        // the tiles' halos wrap once at most: lateral extents of at least 16 nodes
        // (and buffer loads of one shot's volume: under 2^31 bytes)
        const bool use_tiles =
            (w->ndim == 3 && w->nx >= 16 && w->ny >= 16 && S->vol * (int64_t)S->esz < ((int64_t)1 << 31));
        const int64_t tx = (w->nx + kTileX - 1) / kTileX, ty = (w->ny + kTileY - 1) / kTileY;
        for (int64_t i = 0; i < w->nib; ++i) {
          const int code = xyz[i * 4 + 3];
          if (use_tiles && (code == 8 || code == 9) && kTileHalo == 4)
            tiled.push_back((int32_t)i);
          else
            wide.push_back((int32_t)i);
        }
        // lateral tile column, then depth; a tile opens at the first point not covered by the
        // previous one of its column
        auto ckey = [&](int32_t i) { return (int64_t)(xyz[i * 4 + 1] / kTileY) * tx + xyz[i * 4 + 0] / kTileX; };
        std::stable_sort(tiled.begin(), tiled.end(), [&](int32_t a, int32_t b) {
          const int64_t ka = ckey(a), kb = ckey(b);
          return ka != kb ? ka < kb : xyz[a * 4 + 2] < xyz[b * 4 + 2];
        });
        std::vector<int4> tl;
        int zopen = 0;
        for (size_t j = 0; j < tiled.size(); ++j) {
          const int32_t i = tiled[j];
          const int z = xyz[i * 4 + 2];
          if (j == 0 || ckey(i) != ckey(tiled[j - 1]) || z >= zopen + kTileZ || (int)j - tl.back().w >= kTileMaxPoints) {
            zopen = z;
            tl.push_back(make_int4(xyz[i * 4] / kTileX * kTileX, xyz[i * 4 + 1] / kTileY * kTileY, z, (int)j));
          }
        }
        tl.push_back(make_int4(0, 0, 0, (int)tiled.size()));
        S->ntiles = (int)tl.size() - 1;
        S->nwide = (int64_t)wide.size();
        if (S->ntiles > 0 && S->nwide > 0) {
          IB_HIP(hipStreamCreateWithFlags(&S->aux, hipStreamNonBlocking));
          IB_HIP(hipEventCreateWithFlags(&S->ev_fork, hipEventDisableTiming));
          IB_HIP(hipEventCreateWithFlags(&S->ev_join, hipEventDisableTiming));
        }
        int32_t *d_perm = nullptr;
        FreeOnExit<int32_t> free_perm{d_perm};
        if ((s = dalloc(&S->pinfo_t, std::max<size_t>(tiled.size(), 1) * pinfo_dense_bytes(prec))) ||
            (s = dalloc(&S->pinfo_w, std::max<size_t>(wide.size(), 1) * pinfo_bytes(prec))) ||
            (s = dalloc(&S->pinfo_tm, std::max<size_t>(tiled.size(), 1) * pinfo_bytes(prec))) ||
            (s = dalloc_t(&S->tiles, tl.size())) ||
            (s = dalloc_t(&d_perm, std::max<size_t>(std::max(tiled.size(), wide.size()), 1))))
          return fail(s);
        IB_HIP(hipMemcpy(S->tiles, tl.data(), tl.size() * sizeof(int4), hipMemcpyHostToDevice));
        const uint32_t *ro = (prec == IB_F32) ? w->rec_off32 : w->rec_off64;
        if (!tiled.empty()) {
          IB_HIP(hipMemcpy(d_perm, tiled.data(), tiled.size() * 4, hipMemcpyHostToDevice));
          enqueue_make_pinfo_dense(prec, w->ib_xyz, w->dense_first, w->dense_count, w->dense_off, S->scale, d_perm,
                                   (int64_t)tiled.size(), S->pinfo_t, st);
          enqueue_make_pinfo(prec, w->ib_xyz, ro, S->scale, d_perm, (int64_t)tiled.size(), S->pinfo_tm, st);
          if (w->col_off) {
            // column-run records: entry offset and the point's LDS position in its tile
            std::vector<uint32_t> coff(w->nib);
            IB_HIP(hipMemcpy(coff.data(), w->col_off, w->nib * 4, hipMemcpyDeviceToHost));
            std::vector<uint2> cr(tiled.size());
            for (size_t t = 0; t + 1 < tl.size(); ++t)
              for (int j = tl[t].w; j < tl[t + 1].w; ++j) {
                const int32_t i = tiled[j];
                const uint32_t lx = (uint32_t)(xyz[i * 4] - tl[t].x + kTileHalo);
                const uint32_t ly = (uint32_t)(xyz[i * 4 + 1] - tl[t].y + kTileHalo);
                const uint32_t lz = (uint32_t)(xyz[i * 4 + 2] - tl[t].z + kTileHalo);
                cr[j] = make_uint2(coff[i], lx | (ly << 5) | (lz << 10) | (xyz[i * 4 + 3] == 9 ? 0x80000000u : 0u));
              }
            if ((s = dalloc_t(&S->crec, cr.size())) || (s = dalloc(&S->cscale, cr.size() * S->esz))) return fail(s);
            IB_HIP(hipMemcpy(S->crec, cr.data(), cr.size() * sizeof(uint2), hipMemcpyHostToDevice));
            const unsigned nb = (unsigned)((tiled.size() + 255) / 256);
            if (prec == IB_F32)
              hipLaunchKernelGGL(k_gather_scale<float>, dim3(nb), dim3(256), 0, st, (const float *)S->scale, d_perm,
                                 (int64_t)tiled.size(), (float *)S->cscale);
            else
              hipLaunchKernelGGL(k_gather_scale<double>, dim3(nb), dim3(256), 0, st, (const double *)S->scale, d_perm,
                                 (int64_t)tiled.size(), (double *)S->cscale);
            IB_HIP(hipGetLastError());
          }
          IB_HIP(hipStreamSynchronize(st));
        }
        // the tiled patch streams the column-run records (two FP32 shots per pass when the
        // state holds several)
        if (S->crec) S->patch_variant = (prec == IB_F32 && nshots >= 2) ? 9 : 8;
        if (!wide.empty()) {
          IB_HIP(hipMemcpy(d_perm, wide.data(), wide.size() * 4, hipMemcpyHostToDevice));
          enqueue_make_pinfo(prec, w->ib_xyz, ro, S->scale, d_perm, (int64_t)wide.size(), S->pinfo_w, st);
          IB_HIP(hipStreamSynchronize(st));
        }
      }
      enqueue_make_delta(w->ball, (int)w->balls.packed.size(), S->pitch, S->pitch * w->ny, S->delta, st);
      IB_HIP(hipGetLastError());
    }
    IB_HIP(hipStreamSynchronize(st));
    // sources: interior corners only; amplitude factor dt^2 w / (h^d (1 + s))
    std::vector<uint8_t> cls(w->N);
    IB_HIP(hipMemcpy(cls.data(), w->node_class, w->N, hipMemcpyDeviceToHost));
    {
      // planes holding interior nodes, over all columns
      const int64_t nc = w->nx * w->ny;
      int lo = (int)w->nz, hi = 0;
      for (int64_t z = 0; z < w->nz; ++z)
        for (int64_t c = 0; c < nc; ++c)
          if (cls[z * nc + c] & 1) {
            lo = std::min(lo, (int)z);
            hi = std::max(hi, (int)z + 1);
          }
      S->zfirst = lo < hi ? lo : 0;
      S->zlast = lo < hi ? hi : 0;
    }
    if (w->ndim == 3 && w->M == 8) {
      // planes holding interior nodes, per column, then per 64 x TY interior tile
      const int64_t nx = w->nx, ny = w->ny, nz = w->nz;
      std::vector<int> clo(nx * ny, (int)nz), chi(nx * ny, 0);
      for (int64_t z = 0; z < nz; ++z)
        for (int64_t c = 0; c < nx * ny; ++c)
          if (cls[z * nx * ny + c] & 1) {
            clo[c] = std::min(clo[c], (int)z);
            chi[c] = std::max(chi[c], (int)z + 1);
          }
      for (int ty : {16, 32}) {
        const int64_t ntx = (nx + 63) / 64, nty = (ny + ty - 1) / ty;
        std::vector<int2> zr(ntx * nty);
        for (int64_t by = 0; by < nty; ++by)
          for (int64_t bx = 0; bx < ntx; ++bx) {
            int lo = (int)nz, hi = 0;
            for (int64_t y = by * ty; y < std::min(ny, (by + 1) * ty); ++y)
              for (int64_t x = bx * 64; x < std::min(nx, (bx + 1) * 64); ++x) {
                lo = std::min(lo, clo[y * nx + x]);
                hi = std::max(hi, chi[y * nx + x]);
              }
            zr[by * ntx + bx] = make_int2(lo, hi);
          }
        int2 **dst = (ty == 16) ? &S->zrange16 : &S->zrange32;
        if ((s = dalloc_t(dst, zr.size()))) return fail(s);
        IB_HIP(hipMemcpy(*dst, zr.data(), zr.size() * sizeof(int2), hipMemcpyHostToDevice));
      }
    }
    if (w->form == IB_FORM_PV1 && w->ndim == 3) {
      // planes holding interior p or v nodes, per column, then per 64 x 4 column block
      const int64_t nx = w->nx, ny = w->ny, nz = w->nz, nc = nx * ny;
      std::vector<uint8_t> any(cls.size());
      for (size_t q = 0; q < cls.size(); ++q) any[q] = cls[q] & 1;
      std::vector<uint8_t> vc(w->N);
      for (int n = 0; n < 3; ++n) {
        IB_HIP(hipMemcpy(vc.data(), w->vcls[n], w->N, hipMemcpyDeviceToHost));
        for (size_t q = 0; q < vc.size(); ++q) any[q] |= vc[q] & 1;
      }
      std::vector<int> clo(nc, (int)nz), chi(nc, 0);
      for (int64_t z = 0; z < nz; ++z)
        for (int64_t c = 0; c < nc; ++c)
          if (any[z * nc + c]) {
            clo[c] = std::min(clo[c], (int)z);
            chi[c] = std::max(chi[c], (int)z + 1);
          }
      const int64_t nbx = (nx + 63) / 64, nby = (ny + 3) / 4;
      std::vector<int2> zr(nbx * nby);
      for (int64_t by = 0; by < nby; ++by)
        for (int64_t bx = 0; bx < nbx; ++bx) {
          int lo = (int)nz, hi = 0;
          for (int64_t y = by * 4; y < std::min(ny, (by + 1) * 4); ++y)
            for (int64_t x = bx * 64; x < std::min(nx, (bx + 1) * 64); ++x) {
              lo = std::min(lo, clo[y * nx + x]);
              hi = std::max(hi, chi[y * nx + x]);
            }
          zr[by * nbx + bx] = make_int2(lo, hi);
        }
      if ((s = dalloc_t(&S->zr4, zr.size()))) return fail(s);
      IB_HIP(hipMemcpy(S->zr4, zr.data(), zr.size() * sizeof(int2), hipMemcpyHostToDevice));
    }
    std::vector<int64_t> sidx(nshots * 8, -1);
    std::vector<double> swv(nshots * 8, 0.0);
    const double hd = std::pow(w->h, w->ndim);
    // the patch launch may carry the injection only where no source node is an IB point
    // (whose patch row it would race with)
    bool src_at_ib = false;
    for (int sh = 0; sh < nshots; ++sh) {
      int64_t idx[8], idu[8];
      double wt[8];
      if (!corners(w, src_pos + (size_t)sh * w->ndim, idx, wt, S->pitch, true) ||
          !corners(w, src_pos + (size_t)sh * w->ndim, idu, wt, S->pitch, false)) {
        set_error("source %d outside the box", sh);
        return fail(IB_ERR_ARG);
      }
      for (int c = 0; c < 8; ++c) {
        if (idx[c] < 0) continue;
        if (!(cls[idu[c]] & 1)) {
          set_error("source %d touches an exterior node", sh);
          return fail(IB_ERR_ARG);
        }
        if (cls[idu[c]] & 4) src_at_ib = true;
        if (w->form == IB_FORM_PV1 && std::binary_search(S->dnode_h.begin(), S->dnode_h.end(), idx[c]))
          src_at_ib = true;
        int64_t x = idu[c] % w->nx, y = (idu[c] / w->nx) % w->ny, z = idu[c] / (w->nx * w->ny);
        double sd = ax[x] + ay[(w->ndim == 3) ? y : 0] + az[z];
        sidx[sh * 8 + c] = idx[c];
        swv[sh * 8 + c] = (w->form == IB_FORM_PV1 ? dt : dt * dt) * wt[c] / (hd * (1.0 + sd));
      }
    }
    S->io_merge = !src_at_ib && (w->form == IB_FORM_P2 || (S->nrows_g > 0 && S->nrows_d > 0));
    if ((s = dalloc_t(&S->sidx, nshots * 8)) || (s = dalloc(&S->sw, nshots * 8 * S->esz))) return fail(s);
    IB_HIP(hipMemcpy(S->sidx, sidx.data(), nshots * 64, hipMemcpyHostToDevice));
    {
      void *tmp = nullptr;
      std::vector<double> v(swv);
      if ((s = upload_cast(v, &tmp))) return fail(s);
      IB_HIP(hipMemcpy(S->sw, tmp, nshots * 8 * S->esz, hipMemcpyDeviceToDevice));
      dfree(tmp);
    }
    // receivers
    std::vector<int64_t> ridx(std::max(nrec, 1) * 8, -1);
    std::vector<double> rwv(std::max(nrec, 1) * 8, 0.0);
    for (int r = 0; r < nrec; ++r) {
      int64_t idx[8];
      double wt[8];
      if (!corners(w, rec_pos + (size_t)r * w->ndim, idx, wt, S->pitch, true)) {
        set_error("receiver %d outside the box", r);
        return fail(IB_ERR_ARG);
      }
      for (int c = 0; c < 8; ++c) {
        ridx[r * 8 + c] = idx[c];
        rwv[r * 8 + c] = wt[c];
      }
    }
    if ((s = dalloc_t(&S->ridx, ridx.size())) || (s = upload_cast(rwv, &S->rw))) return fail(s);
    S->ridx_h = ridx;
    S->rw_h = rwv;
    IB_HIP(hipMemcpy(S->ridx, ridx.data(), ridx.size() * 8, hipMemcpyHostToDevice));
    if ((s = dalloc_t(&S->tcount, 4))) return fail(s);
    IB_HIP(hipMemset(S->tcount, 0, 32));
    if ((s = dalloc_t(&S->wflag, 2))) return fail(s);
    IB_HIP(hipHostMalloc((void **)&S->wflag_h, 2 * sizeof(int32_t), hipHostMallocDefault));
    IB_HIP(hipEventCreateWithFlags(&S->ev_watch, hipEventDisableTiming));
    watch_reset(S, st);
    IB_HIP(hipGetLastError());
    IB_HIP(hipStreamSynchronize(st));
    // z-chunking of the 3D interior kernel: enough workgroups to fill 256 CUs
    if (w->ndim == 3 && w->form == IB_FORM_P2) {
      int64_t tiles = ((w->nx + 63) / 64) * ((w->ny + 15) / 16) * nshots;
      int64_t want = 2048;
      int nzc = (int)std::max<int64_t>(1, std::min<int64_t>(w->nz / 16, (want + tiles - 1) / tiles));
      S->zchunk = (int)((w->nz + nzc - 1) / nzc);
      S->zchunk_auto = S->zchunk;
      if ((s = autotune_interior(S, st))) return fail(s);
    }
    return IB_OK;
  };
  const ib_status status = build();
  if (status != IB_OK) {
    ib_state_free(S);
    return status;
  }
  *out = S;
  return IB_OK;
}

void ib_state_free(ib_state *S) {
  if (!S) return;
  drop_graphs(S);
  if (S->aux) (void)hipStreamDestroy(S->aux);
  if (S->ev_fork) (void)hipEventDestroy(S->ev_fork);
  if (S->ev_join) (void)hipEventDestroy(S->ev_join);
  dfree(S->buf[0]);
  dfree(S->buf[1]);
  dfree(S->dbuf);
  dfree(S->K);
  dfree(S->sx);
  dfree(S->sy);
  dfree(S->sz);
  dfree(S->scale);
  dfree(S->pinfo);
  dfree(S->pinfo_t);
  dfree(S->pinfo_w);
  dfree(S->pinfo_tm);
  dfree(S->crec);
  dfree(S->cscale);
  dfree(S->tiles);
  dfree(S->zrange16);
  dfree(S->zr4);
  dfree(S->zrange32);
  dfree(S->delta);
  dfree(S->sidx);
  dfree(S->sw);
  dfree(S->ridx);
  dfree(S->rw);
  dfree(S->tcount);
  dfree(S->own.data);
  dfree(S->wflag);
  if (S->wflag_h) (void)hipHostFree(S->wflag_h);
  if (S->ev_watch) (void)hipEventDestroy(S->ev_watch);
  dfree(S->vbuf), dfree(S->kv);
  dfree(S->g_node), dfree(S->g_start), dfree(S->g_enode), dfree(S->d_node), dfree(S->d_start), dfree(S->d_enode);
  dfree(S->g_scale), dfree(S->g_w), dfree(S->d_scale), dfree(S->d_w);
  dfree(S->rnode), dfree(S->roff), dfree(S->rrec);
  dfree(S->jD), dfree(S->ibvals), dfree(S->rD), dfree(S->rwt);
  dfree(S->fF), dfree(S->fs);
  delete S;
}

int64_t ib_state_step_count(const ib_state *S) { return S ? S->t : -1; }

ib_status ib_state_set_tuning(ib_state *S, int32_t variant, int32_t zchunk, int32_t patch_variant) {
  if (!S || zchunk < 0 || variant < 0 || variant > 4 || patch_variant < -1 || patch_variant > 9 ||
      (patch_variant >= 8 && S->ntiles > 0 && !S->crec)) {
    set_error("ib_state_set_tuning: invalid argument");
    return IB_ERR_ARG;
  }
  S->variant = variant;
  if (patch_variant >= 0) S->patch_variant = patch_variant;
  S->zchunk = zchunk > 0 ? zchunk : S->zchunk_auto;
  drop_graphs(S);
  return IB_OK;
}

}  // extern "C"

namespace {

PVArgs make_pv_args(const ib_state *S) {
  const ib_weights *w = S->w;
  PVArgs a{};
  a.prec = S->prec;
  a.ndim = w->ndim;
  a.M = w->M;
  a.nv = S->nv;
  a.nx = (int)w->nx;
  a.ny = (int)w->ny;
  a.nz = (int)w->nz;
  a.pitch = S->pitch;
  a.vol = S->vol;
  a.nshots = S->nshots;
  a.zr4 = S->zr4;
  a.p = S->buf[0];
  a.v = S->vbuf;
  a.kp = S->K;
  a.kv = S->kv;
  for (int n = 0; n < 3; ++n) a.vcls[n] = w->vcls[n];
  a.fv = S->dt / w->h;
  a.sx = S->sx;
  a.sy = S->sy;
  a.sz = S->sz;
  a.nrows_g = S->nrows_g;
  a.nrows_d = S->nrows_d;
  a.g_node = S->g_node, a.g_start = S->g_start, a.g_enode = S->g_enode;
  a.d_node = S->d_node, a.d_start = S->d_start, a.d_enode = S->d_enode;
  a.g_scale = S->g_scale, a.g_w = S->g_w, a.d_scale = S->d_scale, a.d_w = S->d_w;
  a.g_lanes = S->g_lanes;
  a.d_lanes = S->d_lanes;
  return a;
}

// one full step of either form: operator update, source injection, receiver sampling.
// Where the patch (or the first-order rows) launches carry the io, the step's sampling is
// left to the next step (sample_prev) or to flush_sample; returns whether it was.
bool enqueue_full_step(ib_state *S, const void *wavelet, int64_t wstride, void *traces, int64_t trace_nt, int cur,
                       hipStream_t st, bool sample_prev = false) {
  StepArgs a = make_args(S, wavelet, wstride, traces, trace_nt, cur);
  if (S->form == IB_FORM_PV1) {
    PVArgs pa = make_pv_args(S);
    if (S->io_merge) {
      pa.io_merge = 1;
      pa.sample_prev = sample_prev ? 1 : 0;
      pa.sidx = a.sidx;
      pa.sw = a.sw;
      pa.wavelet = a.wavelet;
      pa.wstride = a.wstride;
      pa.ridx = a.ridx;
      pa.rw = a.rw;
      pa.nrec = a.nrec;
      pa.traces = a.traces;
      pa.nsteps = a.nsteps;
      pa.tcount = a.tcount;
      enqueue_pv_step(pa, st);
      return true;
    }
    enqueue_pv_step(pa, st);
    enqueue_source_receivers(a, S->buf[0], st);
    return false;
  }
  a.sample_prev = sample_prev ? 1 : 0;
  enqueue_step(a, st);
  return step_samples_in_patch(a);
}

// the sampling left behind by the last step (its output is the field of parity cur; the
// first-order form keeps p in buf[0])
static void flush_sample(ib_state *S, void *traces, int64_t trace_nt, int cur, hipStream_t st) {
  StepArgs a = make_args(S, nullptr, 0, traces, trace_nt, cur);
  enqueue_sample(a, S->form == IB_FORM_PV1 ? S->buf[0] : S->buf[cur], st);
}

// Watchdog scan of p^n: a wavefront that holds a value outside [-limit, limit] (NaN
// included: it compares false) raises the flag and lowers the recorded step count.
template <typename T>
__global__ void k_watch(const T *__restrict__ p, int64_t n, T limit, int32_t step, int32_t *flag) {
  bool hit = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const T v = p[i];
    hit |= !(v <= limit && v >= -limit);
  }
  if (__any(hit) && (threadIdx.x & (warpSize - 1)) == 0) {
    atomicOr(&flag[0], 1);
    atomicMin(&flag[1], step);
  }
}
__global__ void k_watch_reset(int32_t *flag) {
  if (threadIdx.x == 0) {
    flag[0] = 0;
    flag[1] = INT_MAX;
  }
}
void watch_reset(ib_state *S, hipStream_t st) {
  hipLaunchKernelGGL(k_watch_reset, dim3(1), dim3(64), 0, st, S->wflag);
  S->since_watch = 0;
  S->watch_pending = false;
  S->tripped = false;
  S->trip_step = -1;
}
ib_status watch_scan(ib_state *S, hipStream_t st) {
  const int64_t n = S->vol * S->nshots;
  const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  const int32_t step = (int32_t)std::min<int64_t>(S->t, INT_MAX);
  const void *p = S->buf[S->cur];
  if (S->prec == IB_F32)
    hipLaunchKernelGGL(k_watch<float>, dim3(nb), dim3(256), 0, st, (const float *)p, n,
                       (float)std::min<double>(S->watch_limit, FLT_MAX), step, S->wflag);
  else
    hipLaunchKernelGGL(k_watch<double>, dim3(nb), dim3(256), 0, st, (const double *)p, n,
                       std::min<double>(S->watch_limit, DBL_MAX), step, S->wflag);
  IB_HIP(hipGetLastError());
  IB_HIP(hipMemcpyAsync(S->wflag_h, S->wflag, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  IB_HIP(hipEventRecord(S->ev_watch, st));
  S->watch_pending = true;
  return IB_OK;
}
// Reads the flags of the last scan if it has completed (or waits for it), and refuses the
// call once a scan has seen a bad value.
ib_status watch_poll(ib_state *S, bool wait, const char *who) {
  if (S->watch_pending) {
    const hipError_t e = wait ? hipEventSynchronize(S->ev_watch) : hipEventQuery(S->ev_watch);
    if (e == hipSuccess) {
      S->watch_pending = false;
      if (S->wflag_h[0]) {
        S->tripped = true;
        S->trip_step = S->wflag_h[1];
      }
    } else if (e != hipErrorNotReady) {
      return hip_fail(e, "hipEventQuery(watchdog)", __FILE__, __LINE__);
    }
  }
  if (S->tripped) {
    set_error("%s: the watchdog found a non-finite pressure or one above %g in magnitude after step %lld "
              "(ib_state_set_watchdog clears it)", who, S->watch_limit, (long long)S->trip_step);
    return IB_ERR_NONFINITE;
  }
  return IB_OK;
}

// nsteps steps; traces (may be null) are [nshots][trace_nt][nrec] with step t stored at
// row t - trace_t0.
ib_status run_steps(ib_state *S, int64_t nsteps, const void *wavelet, int64_t wstride, void *traces, int64_t trace_nt,
                    int64_t trace_t0, bool use_graph, hipStream_t st) {
  if (nsteps == 0) return IB_OK;
  hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(1), 0, st, S->tcount, S->t, trace_t0);
  int64_t done = 0;
  if (use_graph && nsteps >= 2) {
    const bool reuse = S->g_wavelet == wavelet && S->g_traces == traces && S->g_wstride == wstride &&
                       S->g_nsteps == trace_nt && S->g_cur == S->cur;
    if (!reuse) drop_graphs(S);
    // the long graph where the call covers it, then the two-step graph
    const int64_t len[2] = {2, kLongGraph};
    for (int k = 1; k >= 0; --k) {
      if (nsteps - done < len[k]) continue;
      if (!S->gexec[k]) {
        hipStream_t cs;
        IB_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        IB_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        bool pending = false;
        for (int64_t q = 0; q < len[k]; ++q)
          pending = enqueue_full_step(S, wavelet, wstride, traces, trace_nt, (int)((S->cur + q) & 1), cs, pending);
        if (pending) flush_sample(S, traces, trace_nt, S->cur, cs);
        hipError_t e = hipStreamEndCapture(cs, &S->graph[k]);
        if (e != hipSuccess) {
          (void)hipStreamDestroy(cs);
          return hip_fail(e, "hipStreamEndCapture", __FILE__, __LINE__);
        }
        (void)hipStreamDestroy(cs);
        IB_HIP(hipGraphInstantiate(&S->gexec[k], S->graph[k], nullptr, nullptr, 0));
        S->g_wavelet = wavelet;
        S->g_traces = traces;
        S->g_wstride = wstride;
        S->g_nsteps = trace_nt;
        S->g_cur = S->cur;
      }
      for (; done + len[k] <= nsteps; done += len[k]) IB_HIP(hipGraphLaunch(S->gexec[k], st));
    }
  }
  bool pending = false;
  for (; done < nsteps; ++done) {
    pending = enqueue_full_step(S, wavelet, wstride, traces, trace_nt, S->cur, st, pending);
    if (S->form == IB_FORM_P2) S->cur ^= 1;
  }
  if (pending) flush_sample(S, traces, trace_nt, S->cur, st);
  IB_HIP(hipGetLastError());
  S->t += nsteps;
  return IB_OK;
}

// run_steps with the watchdog's scan after every watch_every steps (the chunks keep their
// even length, so the captured two-step graph stays valid across them)
ib_status run_steps_watched(ib_state *S, int64_t nsteps, const void *wavelet, int64_t wstride, void *traces,
                            int64_t trace_nt, int64_t trace_t0, bool use_graph, hipStream_t st) {
  if (S->watch_every <= 0) return run_steps(S, nsteps, wavelet, wstride, traces, trace_nt, trace_t0, use_graph, st);
  int64_t done = 0;
  while (done < nsteps) {
    const int64_t n = std::min<int64_t>(nsteps - done, S->watch_every - S->since_watch);
    ib_status s = run_steps(S, n, wavelet, wstride, traces, trace_nt, trace_t0, use_graph, st);
    if (s) return s;
    done += n;
    S->since_watch += n;
    if (S->since_watch >= S->watch_every) {
      S->since_watch = 0;
      if ((s = watch_scan(S, st))) return s;
    }
  }
  return IB_OK;
}

// Transposed IB rows (built on the device once per stencil table and shared by its
// states) with this state's damping factors, and the transposed receivers (host, once per
// state).
template <typename T>
ib_status build_adjoint_tables(ib_state *S, hipStream_t st) {
  // the table is a cache of the (otherwise immutable) stencil table
  ib_weights *w = const_cast<ib_weights *>(S->w);
  const int64_t pitch = S->pitch, ny = w->ny;
  auto Dof = [&](int64_t x, int64_t y, int64_t z) { return 1.0 / (1.0 + S->ax[x] + S->ay[w->ndim == 3 ? y : 0] + S->az[z]); };
  ib_status s;
  if ((s = adjoint_table_build(w, st))) return s;
  S->nj = w->adj_nj;
  if ((s = dalloc(&S->jD, std::max<int64_t>(S->nj, 1) * sizeof(T))) ||
      (s = dalloc(&S->ibvals, std::max<int64_t>(w->nib * S->nshots, 1) * sizeof(T))))
    return s;
  enqueue_adj_D(S->prec, w->adj_jnode, S->nj, S->K, S->sx, S->sy, S->sz, (int)ny, pitch, S->jD, st);
  IB_HIP(hipGetLastError());
  // receivers: node -> (receiver, weight)
  struct RE {
    int64_t j;
    int32_t r;
    double w;
  };
  std::vector<RE> re;
  for (int r = 0; r < S->nrec; ++r)
    for (int c = 0; c < 8; ++c)
      if (S->ridx_h[r * 8 + c] >= 0) re.push_back({S->ridx_h[r * 8 + c], r, S->rw_h[r * 8 + c]});
  std::stable_sort(re.begin(), re.end(), [](const RE &a, const RE &b) { return a.j < b.j; });
  std::vector<int64_t> rn, ro;
  std::vector<int32_t> rr;
  std::vector<T> rd, rwv;
  for (size_t e = 0; e < re.size(); ++e) {
    if (e == 0 || re[e].j != re[e - 1].j) {
      rn.push_back(re[e].j);
      ro.push_back((int64_t)e);
      int64_t j = re[e].j;
      int64_t x = j % pitch, y = (j / pitch) % ny, z = j / (pitch * ny);
      rd.push_back((T)Dof(x, y, z));
    }
    rr.push_back(re[e].r);
    rwv.push_back((T)re[e].w);
  }
  ro.push_back((int64_t)re.size());
  S->nrn = (int64_t)rn.size();
  if ((s = dalloc_t(&S->rnode, std::max<size_t>(rn.size(), 1))) || (s = dalloc_t(&S->roff, ro.size())) ||
      (s = dalloc_t(&S->rrec, std::max<size_t>(rr.size(), 1))) ||
      (s = dalloc(&S->rD, std::max<size_t>(rd.size(), 1) * sizeof(T))) ||
      (s = dalloc(&S->rwt, std::max<size_t>(rwv.size(), 1) * sizeof(T))))
    return s;
  if (!rn.empty()) {
    IB_HIP(hipMemcpy(S->rnode, rn.data(), rn.size() * 8, hipMemcpyHostToDevice));
    IB_HIP(hipMemcpy(S->rrec, rr.data(), rr.size() * 4, hipMemcpyHostToDevice));
    IB_HIP(hipMemcpy(S->rD, rd.data(), rd.size() * sizeof(T), hipMemcpyHostToDevice));
    IB_HIP(hipMemcpy(S->rwt, rwv.data(), rwv.size() * sizeof(T), hipMemcpyHostToDevice));
    // the adjoint runs on mu = K lambda: receiver rows carry K_j / (1 + s_j)
    enqueue_scale_by_K(S->prec, S->rD, S->rnode, (int64_t)rn.size(), S->K, st);
    IB_HIP(hipGetLastError());
    IB_HIP(hipStreamSynchronize(st));
  }
  IB_HIP(hipMemcpy(S->roff, ro.data(), ro.size() * 8, hipMemcpyHostToDevice));
  S->adj_ready = true;
  return IB_OK;
}

// zero a work area with a kernel (stream-ordered, and capturable where a memset is not)
__global__ void k_zero_words(uint32_t *p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}
void zero_bytes(void *p, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 4;
  if (n == 0) return;
  const unsigned nb = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero_words, dim3(nb), dim3(256), 0, st, (uint32_t *)p, n);
}

ib_status adjoint_check(ib_state *S, const ib_checkpoints *C, const void *residual, const void *wavelet,
                        const double *grad, const char *who) {
  if (!S || !C || !residual || !wavelet || !grad || S->form != IB_FORM_P2) {
    set_error("%s: null argument or first-order state", who);
    return IB_ERR_ARG;
  }
  if (C->count == 0 || !C->data) {
    set_error("%s: no checkpoints (run a forward pass first)", who);
    return IB_ERR_STATE;
  }
  if (C->owner != S->uid) {
    set_error("%s: the checkpoints were written by another state", who);
    return IB_ERR_STATE;
  }
  if (ib_status s = watch_poll(S, false, who)) return s;
  if (S->fF) {
    set_error("%s: the state has non-zero boundary values (not differentiated)", who);
    return IB_ERR_STATE;
  }
  return IB_OK;
}

// Work space of one adjoint run: mu^{m+1}, mu^{m+2} (and mu^m - mu^{m+1} in the increment
// form), the recomputed segment (ckpt_every + 2 fields) and the FP64 gradient accumulator,
// each aligned to 256 bytes.
struct AdjLayout {
  size_t lam0, lam1, lamd, seg, gK, total;
};
AdjLayout adjoint_layout(const ib_state *S, const ib_checkpoints *C) {
  const size_t fbytes = (size_t)S->vol * S->nshots * S->esz;
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  AdjLayout L{};
  size_t o = 0;
  L.lam0 = o, o += al(fbytes);
  L.lam1 = o, o += al(fbytes);
  L.lamd = o, o += S->incr ? al(fbytes) : 0;
  L.seg = o, o += al(fbytes * (size_t)(C->every + 2));
  L.gK = o, o += al((size_t)S->vol * sizeof(double));
  L.total = o;
  return L;
}
size_t adjoint_work_bytes(const ib_state *S, const ib_checkpoints *C) { return adjoint_layout(S, C).total; }

// The adjoint sweep over the checkpoint segments, with its work space at ``work`` (at
// least adjoint_work_bytes(S)); enqueued on ``st`` without waiting for it.
ib_status adjoint_run(ib_state *S, const ib_checkpoints *CK, const void *residual, const void *wavelet, int64_t wstride,
                      double *grad, void *work, hipStream_t st) {
  const ib_weights *w = S->w;
  ib_status s;
  const int64_t nt = CK->nt, C = CK->every;
  const size_t fbytes = (size_t)S->vol * S->nshots * S->esz;
  // seg holds u^{t0-1} .. u^{t0+len} of the segment being reversed (C + 2 fields; the
  // increment form keeps d^{t0} .. d^{t0+len}, C + 1 fields); lamd is mu^m - mu^{m+1} of
  // the increment form
  const AdjLayout AL = adjoint_layout(S, CK);
  char *wb = (char *)work;
  void *lam[2] = {wb + AL.lam0, wb + AL.lam1};
  void *lamd = S->incr ? (void *)(wb + AL.lamd) : nullptr;
  void *seg = wb + AL.seg;
  double *gK = (double *)(wb + AL.gK);
  zero_bytes(lam[0], fbytes, st);
  zero_bytes(lam[1], fbytes, st);
  if (lamd) zero_bytes(lamd, fbytes, st);
  zero_bytes(gK, (size_t)S->vol * sizeof(double), st);
  int a1 = 0, a2 = 1;   // lam[a1] = mu^{m+1}, lam[a2] = mu^{m+2}
  auto field = [&](int64_t q) { return (char *)seg + (size_t)q * fbytes; };
  for (int64_t k = CK->count - 1; k >= 0; --k) {
    const int64_t t0 = k * C, len = std::min<int64_t>(C, nt - t0);
    const char *ck = (const char *)CK->data + (size_t)k * 2 * fbytes;
    IB_HIP(hipMemcpyAsync(S->buf[S->cur], ck, fbytes, hipMemcpyDeviceToDevice, st));
    IB_HIP(hipMemcpyAsync(S->incr ? S->dbuf : S->buf[1 - S->cur], ck + fbytes, fbytes, hipMemcpyDeviceToDevice, st));
    S->t = t0;
    if (S->incr) {
      // field(q) = d^{t0+q}
      IB_HIP(hipMemcpyAsync(field(0), ck + fbytes, fbytes, hipMemcpyDeviceToDevice, st));
    } else {
      // field(q) = u^{t0+q-1}
      IB_HIP(hipMemcpyAsync(field(0), ck + fbytes, fbytes, hipMemcpyDeviceToDevice, st));
      IB_HIP(hipMemcpyAsync(field(1), ck, fbytes, hipMemcpyDeviceToDevice, st));
    }
    for (int64_t q = 1; q <= len; ++q) {
      if ((s = run_steps(S, 1, wavelet, wstride, nullptr, 0, 0, false, st))) return s;
      if (S->incr)
        IB_HIP(hipMemcpyAsync(field(q), S->dbuf, fbytes, hipMemcpyDeviceToDevice, st));
      else
        IB_HIP(hipMemcpyAsync(field(q + 1), S->buf[S->cur], fbytes, hipMemcpyDeviceToDevice, st));
    }
    for (int64_t m = t0 + len; m >= t0 + 1; --m) {
      // interior part: the forward interior kernel on mu (mu^{m+2} is overwritten by mu^m)
      StepArgs sa = make_args(S, nullptr, 0, nullptr, 0, S->cur);
      sa.un = lam[a1];
      sa.um = lam[a2];
      sa.dd = lamd;
      enqueue_interior_only(sa, st);
      AdjArgs a{};
      a.prec = S->prec;
      a.ndim = w->ndim;
      a.M = w->M;
      a.nx = (int)w->nx;
      a.ny = (int)w->ny;
      a.nz = (int)w->nz;
      a.pitch = S->pitch;
      a.vol = S->vol;
      a.nshots = S->nshots;
      a.lam1 = lam[a1];
      a.lam2 = lam[a2];
      a.lamd = lamd;
      a.K = S->K;
      a.sx = S->sx;
      a.sy = S->sy;
      a.sz = S->sz;
      a.nj = S->nj;
      a.jnode = w->adj_jnode;
      a.joff = w->adj_joff;
      a.jsrc = w->adj_jsrc;
      a.jD = S->jD;
      a.jw = (S->prec == IB_F32) ? (const void *)w->adj_jw32 : (const void *)w->adj_jw64;
      a.ibxyz = w->ib_xyz;
      a.vals = S->ibvals;
      a.nib = w->nib;
      a.nrn = S->nrn;
      a.rnode = S->rnode;
      a.roff = S->roff;
      a.rrec = S->rrec;
      a.rD = S->rD;
      a.rw = S->rwt;
      a.res = residual;
      a.nt = nt;
      a.nrec = S->nrec;
      a.step = m - 1;
      a.gK = gK;
      if (S->incr) {
        a.u2 = field(m - t0);       // d^m
        a.u1 = nullptr;
        a.u0 = field(m - t0 - 1);   // d^{m-1}
      } else {
        a.u2 = field(m - t0 + 1);   // u^m
        a.u1 = field(m - t0);       // u^{m-1}
        a.u0 = field(m - t0 - 1);   // u^{m-2}
      }
      a.sidx = S->sidx;
      a.sw = S->sw;
      a.wavelet = wavelet;
      a.wstride = wstride;
      enqueue_adjoint_step(a, st);
      std::swap(a1, a2);
    }
  }
  enqueue_grad_out(S->prec, gK, S->K, grad, (int)w->nx, (int)w->ny, (int)w->nz, S->pitch, S->dt / w->h, st);
  IB_HIP(hipGetLastError());
  // the wavefields now hold the recomputed first segment; the step counter follows them
  return IB_OK;
}

// The adjoint on a freshly allocated work space, released once the stream has used it.
ib_status adjoint_alloc(ib_state *S, const ib_checkpoints *C, const void *residual, const void *wavelet,
                        int64_t wstride, double *grad, hipStream_t st, const char *who) {
  ib_status s = adjoint_check(S, C, residual, wavelet, grad, who);
  if (s) return s;
  if (!S->adj_ready) {
    s = (S->prec == IB_F32) ? build_adjoint_tables<float>(S, st) : build_adjoint_tables<double>(S, st);
    if (s) return s;
  }
  void *work = nullptr;
  if ((s = dalloc(&work, adjoint_work_bytes(S, C)))) return s;
  s = adjoint_run(S, C, residual, wavelet, wstride, grad, work, st);
  const hipError_t e = hipStreamSynchronize(st);
  dfree(work);
  if (s) return s;
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize", __FILE__, __LINE__);
  return IB_OK;
}

// Forward modelling from rest into the checkpoint set C (reallocated when its size changes).
ib_status forward_into(ib_state *S, ib_checkpoints *C, int32_t nt, const void *wavelet, int64_t wstride, void *traces,
                       int32_t ckpt_every, hipStream_t st, const char *who) {
  if (!S || !C || nt < 1 || !wavelet || ckpt_every < 1 || wstride < nt || (S->nrec > 0 && !traces) ||
      S->form != IB_FORM_P2) {
    set_error("%s: invalid argument", who);
    return IB_ERR_ARG;
  }
  if (S->fF) {
    set_error("%s: the state has non-zero boundary values (not differentiated by the adjoint)", who);
    return IB_ERR_STATE;
  }
  if (ib_status s = watch_poll(S, false, who)) return s;
  const size_t fbytes = (size_t)S->vol * S->nshots * S->esz;
  const int64_t nck = (nt + ckpt_every - 1) / ckpt_every;
  if (C->bytes != 2 * fbytes * nck || !C->data) {
    dfree(C->data);
    C->data = nullptr;
    C->bytes = 0;
    C->count = 0;
    ib_status s = dalloc(&C->data, 2 * fbytes * nck);
    if (s) return s;
    C->bytes = 2 * fbytes * nck;
  }
  C->owner = S->uid;
  C->count = nck;
  C->nt = nt;
  C->every = ckpt_every;
  // the adjoint's transposed tables are built here, so that an adjoint call can run on
  // memory that exists already
  if (!S->adj_ready) {
    ib_status s = (S->prec == IB_F32) ? build_adjoint_tables<float>(S, st) : build_adjoint_tables<double>(S, st);
    if (s) return s;
  }
  IB_HIP(hipMemsetAsync(S->buf[0], 0, fbytes, st));
  IB_HIP(hipMemsetAsync(S->buf[1], 0, fbytes, st));
  if (S->incr) IB_HIP(hipMemsetAsync(S->dbuf, 0, fbytes, st));
  S->t = 0;
  S->since_watch = 0;
  for (int64_t k = 0; k < nck; ++k) {
    // checkpoint k: p^n and p^{n-1} (plain form) or d^n (increment form)
    char *ck = (char *)C->data + (size_t)k * 2 * fbytes;
    IB_HIP(hipMemcpyAsync(ck, S->buf[S->cur], fbytes, hipMemcpyDeviceToDevice, st));
    IB_HIP(hipMemcpyAsync(ck + fbytes, S->incr ? S->dbuf : S->buf[1 - S->cur], fbytes, hipMemcpyDeviceToDevice, st));
    int64_t n = std::min<int64_t>(ckpt_every, nt - k * ckpt_every);
    ib_status s = run_steps_watched(S, n, wavelet, wstride, traces, nt, 0, false, st);
    if (s) return s;
  }
  return IB_OK;
}

}  // namespace

extern "C" {

ib_status ib_step(ib_state *S, int32_t nsteps, const void *wavelet, int64_t wstride, void *traces, int32_t use_graph,
                  void *stream) {
  if (!S || nsteps < 0 || (S->nrec > 0 && nsteps > 0 && !traces) || !wavelet) {
    set_error("ib_step: invalid argument");
    return IB_ERR_ARG;
  }
  if (S->t + nsteps > wstride) {
    set_error("ib_step: wavelet has %lld samples, steps up to %lld requested", (long long)wstride,
              (long long)(S->t + nsteps));
    return IB_ERR_ARG;
  }
  if (S->fF && S->t + nsteps > S->flen) {
    set_error("ib_step: boundary-value time functions have %lld samples, steps up to %lld requested",
              (long long)S->flen, (long long)(S->t + nsteps));
    return IB_ERR_ARG;
  }
  if (ib_status s = watch_poll(S, false, "ib_step")) return s;
  return run_steps_watched(S, nsteps, wavelet, wstride, traces, nsteps, S->t, use_graph != 0, (hipStream_t)stream);
}

ib_status ib_forward(ib_state *S, int32_t nt, const void *wavelet, int64_t wstride, void *traces, int32_t ckpt_every,
                     void *stream) {
  return forward_into(S, S ? &S->own : nullptr, nt, wavelet, wstride, traces, ckpt_every, (hipStream_t)stream,
                      "ib_forward");
}

ib_status ib_forward_ckpt(ib_state *S, int32_t nt, const void *wavelet, int64_t wstride, void *traces,
                          int32_t ckpt_every, ib_checkpoints **ckpt, void *stream) {
  if (!ckpt) {
    set_error("ib_forward_ckpt: null checkpoint handle pointer");
    return IB_ERR_ARG;
  }
  ib_checkpoints *C = *ckpt;
  const bool fresh = (C == nullptr);
  if (fresh) C = new ib_checkpoints();
  const ib_status s = forward_into(S, C, nt, wavelet, wstride, traces, ckpt_every, (hipStream_t)stream,
                                   "ib_forward_ckpt");
  if (s != IB_OK) {
    if (fresh) ib_checkpoints_free(C);
    return s;
  }
  *ckpt = C;
  return IB_OK;
}

void ib_checkpoints_free(ib_checkpoints *C) {
  if (!C) return;
  dfree(C->data);
  delete C;
}

ib_status ib_adjoint_ckpt(ib_state *S, const ib_checkpoints *C, const void *residual, const void *wavelet,
                          int64_t wstride, double *grad, void *stream) {
  return adjoint_alloc(S, C, residual, wavelet, wstride, grad, (hipStream_t)stream, "ib_adjoint_ckpt");
}

ib_status ib_adjoint(ib_state *S, const void *residual, const void *wavelet, int64_t wstride, double *grad,
                     void *stream) {
  return adjoint_alloc(S, S ? &S->own : nullptr, residual, wavelet, wstride, grad, (hipStream_t)stream, "ib_adjoint");
}

}  // extern "C"

namespace {
// Work space of ib_adjoint_noalloc: a fixed device array (each device that runs it holds its
// own copy until the process ends).  Host code never uses its name as an address: the
// address comes from hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

ib_status scratch_address(void **out) {
  int dev = 0;
  IB_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("ib_adjoint_noalloc: device %d beyond the %d the work space table covers", dev, kMaxDevices);
    return IB_ERR_ARG;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return IB_OK;
}
}  // namespace

extern "C" {

ib_status ib_adjoint_noalloc(ib_state *S, const void *residual, const void *wavelet, int64_t wstride, double *grad,
                             void *stream) {
  ib_status s = adjoint_check(S, S ? &S->own : nullptr, residual, wavelet, grad, "ib_adjoint_noalloc");
  if (s) return s;
  if (!S->adj_ready) {
    set_error("ib_adjoint_noalloc: the adjoint tables are missing (call ib_forward first)");
    return IB_ERR_STATE;
  }
  const size_t need = adjoint_work_bytes(S, &S->own);
  if (need > kScratchBytes) {
    set_error("ib_adjoint_noalloc: this state needs %zu bytes of work space, more than the %zu available "
              "(fewer shots, a smaller grid or a shorter checkpoint interval fit; ib_adjoint has no limit)",
              need, kScratchBytes);
    return IB_ERR_ARG;
  }
  void *work = nullptr;
  if ((s = scratch_address(&work))) return s;
  return adjoint_run(S, &S->own, residual, wavelet, wstride, grad, work, (hipStream_t)stream);
}

ib_status ib_state_set_watchdog(ib_state *S, int32_t every, double limit, void *stream) {
  if (!S || every < 0 || !(limit > 0.0)) {
    set_error("ib_state_set_watchdog: invalid argument");
    return IB_ERR_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  // a scan still in flight is waited for, so that its flags cannot come back after the reset
  if (S->watch_pending) IB_HIP(hipEventSynchronize(S->ev_watch));
  S->watch_every = every + (every & 1);
  S->watch_limit = limit;
  watch_reset(S, st);
  IB_HIP(hipGetLastError());
  return IB_OK;
}

ib_status ib_state_status(ib_state *S, int32_t wait) {
  if (!S) {
    set_error("ib_state_status: null state");
    return IB_ERR_ARG;
  }
  return watch_poll(S, wait != 0, "ib_state_status");
}

ib_status ib_state_run_kernel(ib_state *S, int32_t which, int32_t count, void *stream) {
  if (!S || which < 0 || which > 1 || count < 0 || S->form != IB_FORM_P2) {
    set_error("ib_state_run_kernel: invalid argument");
    return IB_ERR_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  for (int i = 0; i < count; ++i) {
    StepArgs a = make_args(S, nullptr, 0, nullptr, 0, S->cur);
    if (which == 0) {
      enqueue_interior_only(a, st);
      S->cur ^= 1;
    } else {
      enqueue_patch_only(a, st);
    }
  }
  IB_HIP(hipGetLastError());
  return IB_OK;
}


ib_status ib_state_set_forcing(ib_state *S, const double *g, int32_t nq, const double *s_host, int64_t s_len,
                               void *stream) {
  if (!S) {
    set_error("ib_state_set_forcing: null state");
    return IB_ERR_ARG;
  }
  const ib_weights *w = S->w;
  if (S->form != IB_FORM_P2) {
    set_error("ib_state_set_forcing: boundary values are supported for the second-order form only");
    return IB_ERR_STATE;
  }
  hipStream_t st = (hipStream_t)stream;
  // the captured graph holds the old pointers
  drop_graphs(S);
  if (!g) {
    IB_HIP(hipStreamSynchronize(st));
    dfree(S->fF), dfree(S->fs);
    S->fF = S->fs = nullptr;
    S->fnq = 0;
    S->flen = 0;
    return IB_OK;
  }
  if (!w->bc_off) {
    set_error("ib_state_set_forcing: the weights were built without condition-value weights (keep_bc_weights = 0)");
    return IB_ERR_STATE;
  }
  if (nq < 1 || nq > w->bc_nq || !s_host || s_len < 1) {
    set_error("ib_state_set_forcing: need 1 <= nq <= %d, a time function and s_len >= 1", w->bc_nq);
    return IB_ERR_ARG;
  }
  IB_HIP(hipStreamSynchronize(st));
  dfree(S->fF), dfree(S->fs);
  S->fF = S->fs = nullptr;
  S->fnq = 0;
  S->flen = 0;
  ib_status s;
  void *F = nullptr, *fs = nullptr;
  if ((s = dalloc(&F, (size_t)std::max<int64_t>(w->nib, 1) * nq * S->esz)) ||
      (s = dalloc(&fs, (size_t)nq * s_len * S->esz))) {
    dfree(F);
    return s;
  }
  std::vector<char> hs((size_t)nq * s_len * S->esz);
  for (int64_t k = 0; k < (int64_t)nq * s_len; ++k) {
    if (S->prec == IB_F32)
      ((float *)hs.data())[k] = (float)s_host[k];
    else
      ((double *)hs.data())[k] = s_host[k];
  }
  IB_HIP(hipMemcpy(fs, hs.data(), hs.size(), hipMemcpyHostToDevice));
  HPow hp{};
  const bool rigid = w->prm.surface == IB_SURF_RIGID;   // free and robin members have order 2q in g
  for (int q = 0; q < 8; ++q) hp.v[q] = std::pow(w->h, rigid ? 2 * q + 1 : 2 * q);
  if (w->nib) {
    const unsigned nb = (unsigned)((w->nib + 255) / 256);
    if (S->prec == IB_F32)
      hipLaunchKernelGGL(k_forcing_setup<float>, dim3(nb), dim3(256), 0, st, w->nib, w->bc_off, w->bc_cnt, w->bc_idx,
                         w->bc_w, g, nq, hp, (const float *)S->scale, (float *)F);
    else
      hipLaunchKernelGGL(k_forcing_setup<double>, dim3(nb), dim3(256), 0, st, w->nib, w->bc_off, w->bc_cnt,
                         w->bc_idx, w->bc_w, g, nq, hp, (const double *)S->scale, (double *)F);
    IB_HIP(hipGetLastError());
  }
  IB_HIP(hipStreamSynchronize(st));
  S->fF = F;
  S->fs = fs;
  S->fnq = nq;
  S->flen = s_len;
  return IB_OK;
}

ib_status ib_state_field(ib_state *S, int32_t which, int32_t shot, void *dev, int32_t direction, void *stream) {
  const int maxw = (S && S->form == IB_FORM_PV1) ? 1 + S->nv : 1;
  if (!S || !dev || which < 0 || which > maxw || shot < 0 || shot >= S->nshots || direction < 0 || direction > 1 ||
      (S->form == IB_FORM_PV1 && which == 1)) {
    set_error("ib_state_field: invalid argument");
    return IB_ERR_ARG;
  }
  const ib_weights *w = S->w;
  const size_t so = (size_t)shot * S->vol * S->esz;
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = w->nx * w->ny * w->nz;
  const dim3 g((unsigned)((n + 255) / 256)), b(256);
  const int nx = (int)w->nx, ny = (int)w->ny, nz = (int)w->nz;
  if (S->incr && which == 1) {
    // the state keeps d^n = p^n - p^{n-1}
    char *p = (char *)S->buf[S->cur] + so, *d = (char *)S->dbuf + so;
    if (S->prec == IB_F32)
      hipLaunchKernelGGL(k_field_prev<float>, g, b, 0, st, (const float *)p, (float *)d, (float *)dev,
                         (const float *)S->K, nx, ny, nz, S->pitch, direction);
    else
      hipLaunchKernelGGL(k_field_prev<double>, g, b, 0, st, (const double *)p, (double *)d, (double *)dev,
                         (const double *)S->K, nx, ny, nz, S->pitch, direction);
    IB_HIP(hipGetLastError());
    return IB_OK;
  }
  char *base;
  const void *mask;
  if (S->form == IB_FORM_PV1) {
    base = (which == 0) ? (char *)S->buf[0] + so : (char *)S->vbuf + ((size_t)shot * S->nv + (which - 2)) * S->vol * S->esz;
    mask = (which == 0) ? S->K : (const char *)S->kv + (size_t)(which - 2) * S->vol * S->esz;
  } else {
    base = (char *)S->buf[which == 0 ? S->cur : 1 - S->cur] + so;
    mask = S->K;
  }
  size_t rowb = w->nx * S->esz, pitchb = S->pitch * S->esz;
  size_t rows = w->ny * w->nz;
  if (direction == 0) {
    IB_HIP(hipMemcpy2DAsync(dev, rowb, base, pitchb, rowb, rows, hipMemcpyDeviceToDevice, st));
  } else {
    IB_HIP(hipMemcpy2DAsync(base, pitchb, dev, rowb, rowb, rows, hipMemcpyDeviceToDevice, st));
    if (S->prec == IB_F32)
      hipLaunchKernelGGL(k_mask_field<float>, g, b, 0, st, (float *)base, (const float *)mask, nx, ny, nz, S->pitch);
    else
      hipLaunchKernelGGL(k_mask_field<double>, g, b, 0, st, (double *)base, (const double *)mask, nx, ny, nz,
                         S->pitch);
    IB_HIP(hipGetLastError());
  }
  return IB_OK;
}

}  // extern "C"
