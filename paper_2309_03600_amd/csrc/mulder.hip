// Per-axis 1D extrapolation table (the reduction to 1D of the method; second-order form,
// free surface).
//
// For an IB point, each side of each axis stencil that reaches an exterior node is
// continued by one polynomial along the axis line.  With the free-surface conditions
// p = p'' = ... = p^(M) = 0 where the line crosses the surface (at distance t_b), the
// polynomial of degree M reduces to its odd part in tau = t - t_b,
//   p(tau) = a_1 tau + a_3 tau^3 + ... + a_{M-1} tau^{M-1},
// fitted exactly to the M/2 interior nodes of the line nearest the crossing and farther
// than eta from it.  The value at an exterior node e is then v_e^T V^{-1} u with
// V_jm = tau_j^(2m-1), so its weights on the data nodes are x = V^{-T} v_e; scaled by the
// interior stencil's weight for e they form the point's modified row, stored in the same
// compact records as the N-D table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ib_internal.h"
#include "surface.h"

namespace ib {

namespace {

constexpr int kMaxHalf = kMaxOrder / 2;

// Solve V^T x = v for a k x k matrix V (k <= kMaxHalf) by Gaussian elimination with
// partial pivoting; false when V is singular.
__device__ bool solve_t(double V[kMaxHalf][kMaxHalf], const double *v, double *x, int k) {
  double A[kMaxHalf][kMaxHalf + 1];
  for (int i = 0; i < k; ++i) {
    for (int j = 0; j < k; ++j) A[i][j] = V[j][i];
    A[i][k] = v[i];
  }
  for (int c = 0; c < k; ++c) {
    int p = c;
    for (int r = c + 1; r < k; ++r)
      if (fabs(A[r][c]) > fabs(A[p][c])) p = r;
    if (!(fabs(A[p][c]) > 0.0)) return false;
    if (p != c)
      for (int j = 0; j <= k; ++j) {
        const double t = A[c][j];
        A[c][j] = A[p][j];
        A[p][j] = t;
      }
    for (int r = c + 1; r < k; ++r) {
      const double f = A[r][c] / A[c][c];
      for (int j = c; j <= k; ++j) A[r][j] -= f * A[c][j];
    }
  }
  for (int r = k - 1; r >= 0; --r) {
    double s = A[r][k];
    for (int j = r + 1; j < k; ++j) s -= A[r][j] * x[j];
    x[r] = s / A[r][r];
  }
  return true;
}

struct Mulder1DArgs {
  SurfView sv;
  const uint8_t *cls;
  const int64_t *ib_node;
  int64_t nib;
  int nx, ny, nz, ndim, M;
  double eta, sgn_phys;
  double w2[2 * kMaxOrder + 1];   // interior second-derivative weights, offsets -M/2..M/2
  int emax;
  int32_t *eoff;                  // [nib][emax] packed offsets (dx, dy, dz as bytes)
  double *ew;                     // [nib][emax]
  int32_t *ecount;                // [nib]
  int32_t *status;                // [nib]: 1 ok, 0 line leaves the interior, -1 singular
};

// one thread per IB point
__global__ void k_mulder(Mulder1DArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.nib) return;
  const int64_t node = a.ib_node[i];
  const int x = (int)(node % a.nx);
  const int64_t r = node / a.nx;
  const int y = (int)(r % a.ny), z = (int)(r / a.ny);
  const int half = a.M / 2, depth = a.ndim - 1;
  int ne = 0, st = 1;
  int32_t *eo = a.eoff + i * a.emax;
  double *ew = a.ew + i * a.emax;
  auto cls_at = [&](int axis, int t, bool &inbox) -> uint8_t {
    int xx = x, yy = y, zz = z;
    if (axis == depth) zz += t;
    else if (axis == 0) xx = wrapi(x + t, a.nx);
    else yy = wrapi(y + t, a.ny);
    inbox = zz >= 0 && zz < a.nz;
    return inbox ? a.cls[((int64_t)zz * a.ny + yy) * a.nx + xx] : (uint8_t)0;
  };
  for (int axis = 0; axis < a.ndim && st == 1; ++axis) {
    for (int sgn = 1; sgn >= -1 && st == 1; sgn -= 2) {
      int k = 0;
      for (int t = 1; t <= half && !k; ++t) {
        bool inbox;
        const uint8_t c = cls_at(axis, sgn * t, inbox);
        if (inbox && !(c & 1)) k = t;
      }
      if (!k) continue;
      // crossing of the line with the surface, t_b in (k-1, k]
      double tb;
      if (axis == depth) {
        tb = sgn * (a.sv.Hs[(size_t)y * a.nx + x] - z);
      } else {
        double lo = k - 1, hi = k;
        for (int it = 0; it < 200; ++it) {
          const double m = 0.5 * (lo + hi);
          if (m <= lo || m >= hi) break;
          double H, g[2], hh[3];
          surf_eval(a.sv, x + (axis == 0 ? sgn * m : 0.0), y + (axis == 1 ? sgn * m : 0.0), H, g, hh);
          if (a.sgn_phys * (z - H) > 0.0)
            lo = m;
          else
            hi = m;
        }
        tb = 0.5 * (lo + hi);
      }
      // the M/2 interior nodes of the line nearest the crossing, farther than eta
      double tau[kMaxHalf];
      int toff[kMaxHalf];
      int nd = 0;
      for (int t = k - 1; nd < half; --t) {
        bool inbox;
        const uint8_t c = cls_at(axis, sgn * t, inbox);
        if (!inbox || !(c & 1)) {
          st = 0;
          break;
        }
        if (tb - t > a.eta) {
          tau[nd] = t - tb;
          toff[nd] = sgn * t;
          ++nd;
        }
      }
      if (st != 1) break;
      double V[kMaxHalf][kMaxHalf];
      for (int j = 0; j < half; ++j) {
        double p = tau[j];
        const double t2 = tau[j] * tau[j];
        for (int m = 0; m < half; ++m) {
          V[j][m] = p;
          p *= t2;
        }
      }
      for (int e = k; e <= half && st == 1; ++e) {
        bool inbox;
        const uint8_t c = cls_at(axis, sgn * e, inbox);
        if (!inbox || (c & 1)) continue;             // interior again: its own value is used
        double v[kMaxHalf], xw[kMaxHalf];
        const double te = e - tb, t2 = te * te;
        double p = te;
        for (int m = 0; m < half; ++m) {
          v[m] = p;
          p *= t2;
        }
        if (!solve_t(V, v, xw, half)) {
          st = -1;
          break;
        }
        const double we = a.w2[sgn * e + half];
        for (int j = 0; j < half; ++j) {
          int d[3] = {0, 0, 0};
          d[axis == depth ? 2 : axis] = toff[j];
          const int32_t packed = (int32_t)((uint32_t)(uint8_t)(int8_t)d[0] | ((uint32_t)(uint8_t)(int8_t)d[1] << 8) |
                                           ((uint32_t)(uint8_t)(int8_t)d[2] << 16));
          if (ne < a.emax) {
            eo[ne] = packed;
            ew[ne] = we * xw[j];
          }
          ++ne;
        }
      }
    }
  }
  if (st == 1 && ne > a.emax) st = -2;
  a.ecount[i] = ne;
  a.status[i] = st;
}

}  // namespace

ib_status mulder_build(ib_weights *w, hipStream_t st) {
  const int ndim = w->ndim, M = w->M, half = M / 2;
  const int64_t nib = w->nib;
  // every point uses the ball of radius M/2 + 1.5: the data nodes lie on the axis lines
  // within M/2 + 1 cells (one node may be skipped for eta)
  const int code = M + 3;
  w->max_code = std::max(M + 1 + 2 * w->prm.max_radius_steps, code);
  ib_status s;
  if ((s = upload_ball_tables(w, st))) return s;
  const int emax = 2 * ndim * half * half;
  Mulder1DArgs a{};
  a.sv = SurfView{w->Hs, (int)w->nx, (int)w->ny, ndim - 1};
  a.cls = w->node_class;
  a.ib_node = w->ib_node;
  a.nib = nib;
  a.nx = (int)w->nx;
  a.ny = (int)w->ny;
  a.nz = (int)w->nz;
  a.ndim = ndim;
  a.M = M;
  a.eta = w->prm.eta;
  a.sgn_phys = w->prm.physical_below ? 1.0 : -1.0;
  second_derivative_weights(M, a.w2);
  a.emax = emax;
  if ((s = dalloc_t(&a.eoff, std::max<int64_t>(nib * emax, 1))) || (s = dalloc_t(&a.ew, std::max<int64_t>(nib * emax, 1))) ||
      (s = dalloc_t(&a.ecount, std::max<int64_t>(nib, 1))) || (s = dalloc_t(&a.status, std::max<int64_t>(nib, 1))))
    return s;
  if (nib)
    hipLaunchKernelGGL(k_mulder, dim3((unsigned)((nib + 127) / 128)), dim3(128), 0, st, a);
  IB_HIP(hipGetLastError());
  std::vector<int32_t> eo(nib * emax), cnt(nib), stat(nib);
  std::vector<double> ewv(nib * emax);
  std::vector<int64_t> hnode(nib);
  if (nib) {
    IB_HIP(hipMemcpyAsync(eo.data(), a.eoff, eo.size() * 4, hipMemcpyDeviceToHost, st));
    IB_HIP(hipMemcpyAsync(ewv.data(), a.ew, ewv.size() * 8, hipMemcpyDeviceToHost, st));
    IB_HIP(hipMemcpyAsync(cnt.data(), a.ecount, nib * 4, hipMemcpyDeviceToHost, st));
    IB_HIP(hipMemcpyAsync(stat.data(), a.status, nib * 4, hipMemcpyDeviceToHost, st));
    IB_HIP(hipMemcpyAsync(hnode.data(), w->ib_node, nib * 8, hipMemcpyDeviceToHost, st));
  }
  IB_HIP(hipStreamSynchronize(st));
  dfree(a.eoff), dfree(a.ew), dfree(a.ecount), dfree(a.status);
  for (int64_t i = 0; i < nib; ++i)
    if (stat[i] != 1) {
      set_error("IB point at node %lld: 1D extrapolation impossible (%s)", (long long)hnode[i],
                stat[i] == 0 ? "the axis line leaves the interior before M/2 data nodes" : "singular line system");
      return IB_ERR_UNCONSTRAINED;
    }
  // lattice index of each offset in the ball of this code
  const int R = code / 2 + 1, side = 2 * R + 1;
  std::vector<int32_t> lut((size_t)side * side * side, -1);
  const int st0 = w->balls.start[code], nb = w->balls.count[code];
  for (int b = 0; b < nb; ++b) {
    const uint32_t v = (uint32_t)w->balls.packed[st0 + b];
    const int dx = (int8_t)(v & 255), dy = (int8_t)((v >> 8) & 255), dz = (int8_t)((v >> 16) & 255);
    lut[((size_t)(dz + R) * side + (dy + R)) * side + (dx + R)] = b;
  }
  const int nwords = (nb + 31) / 32, nwords64 = (nwords + 1) & ~1;
  std::vector<double> w64;
  std::vector<uint32_t> rec32, rec64, roff32(nib), roff64(nib);
  std::vector<int16_t> xyz(nib * 4);
  std::vector<int32_t> meta(nib * 4);
  std::vector<double> acc(nb);
  std::vector<uint8_t> on(nb);
  int64_t maxnw = 0;
  for (int64_t i = 0; i < nib; ++i) {
    std::fill(acc.begin(), acc.end(), 0.0);
    std::fill(on.begin(), on.end(), 0);
    for (int q = 0; q < cnt[i]; ++q) {
      const uint32_t v = (uint32_t)eo[i * emax + q];
      const int dx = (int8_t)(v & 255), dy = (int8_t)((v >> 8) & 255), dz = (int8_t)((v >> 16) & 255);
      const int b = lut[((size_t)(dz + R) * side + (dy + R)) * side + (dx + R)];
      if (b < 0) {
        set_error("1D extrapolation: data node outside the support ball");
        return IB_ERR_ARG;
      }
      acc[b] += ewv[i * emax + q];
      on[b] = 1;
    }
    std::vector<uint32_t> mask(nwords, 0u);
    int nw = 0;
    for (int b = 0; b < nb; ++b)
      if (on[b]) {
        mask[b >> 5] |= 1u << (b & 31);
        ++nw;
      }
    const int64_t node = hnode[i];
    xyz[i * 4] = (int16_t)(node % w->nx);
    xyz[i * 4 + 1] = (int16_t)((node / w->nx) % w->ny);
    xyz[i * 4 + 2] = (int16_t)(node / (w->nx * w->ny));
    xyz[i * 4 + 3] = (int16_t)code;
    meta[i * 4] = 0;
    meta[i * 4 + 1] = M;
    meta[i * 4 + 2] = nw;
    meta[i * 4 + 3] = (int32_t)w64.size();
    roff32[i] = (uint32_t)rec32.size();
    roff64[i] = (uint32_t)rec64.size();
    rec32.insert(rec32.end(), mask.begin(), mask.end());
    rec64.insert(rec64.end(), mask.begin(), mask.end());
    if (nwords64 > nwords) rec64.push_back(0u);
    for (int b = 0; b < nb; ++b)
      if (on[b]) {
        const double v = acc[b];
        w64.push_back(v);
        const float f = (float)v;
        uint32_t u32;
        std::memcpy(&u32, &f, 4);
        rec32.push_back(u32);
        uint64_t u64;
        std::memcpy(&u64, &v, 8);
        rec64.push_back((uint32_t)(u64 & 0xffffffffu));
        rec64.push_back((uint32_t)(u64 >> 32));
      }
    maxnw = std::max<int64_t>(maxnw, nw);
  }
  w->sumw = (int64_t)w64.size();
  w->rec32_words = (int64_t)rec32.size();
  w->rec64_words = (int64_t)rec64.size();
  w->stats.sum_nw = w->sumw;
  w->stats.max_nw = maxnw;
  w->stats.max_cond = 0.0;
  w->stats.min_margin = 0.0;
  w->stats.table_bytes_f32 = w->rec32_words * 4;
  w->stats.table_bytes_f64 = w->rec64_words * 4;
  w->stats.max_ball = nb;
  w->stats.radius_hist[0] = nib;
  w->stats.order_hist[std::min(M, 16)] = nib;
  std::vector<double> sig(nib, 1.0);
  if ((s = dalloc_t(&w->w64, std::max<int64_t>(w->sumw, 1))) ||
      (s = dalloc_t(&w->rec32, std::max<int64_t>(w->rec32_words, 1))) ||
      (s = dalloc_t(&w->rec64, std::max<int64_t>(w->rec64_words, 1))) ||
      (s = dalloc_t(&w->rec_off32, std::max<int64_t>(nib, 1))) || (s = dalloc_t(&w->rec_off64, std::max<int64_t>(nib, 1))) ||
      (s = dalloc_t(&w->ib_xyz, std::max<int64_t>(nib, 1) * 4)) || (s = dalloc_t(&w->ib_meta, std::max<int64_t>(nib, 1) * 4)) ||
      (s = dalloc_t(&w->ib_sigma, std::max<int64_t>(nib, 1))))
    return s;
  if (nib) {
    IB_HIP(hipMemcpy(w->w64, w64.data(), w64.size() * 8, hipMemcpyHostToDevice));
    IB_HIP(hipMemcpy(w->rec32, rec32.data(), rec32.size() * 4, hipMemcpyHostToDevice));
    IB_HIP(hipMemcpy(w->rec64, rec64.data(), rec64.size() * 4, hipMemcpyHostToDevice));
    IB_HIP(hipMemcpy(w->rec_off32, roff32.data(), nib * 4, hipMemcpyHostToDevice));
    IB_HIP(hipMemcpy(w->rec_off64, roff64.data(), nib * 4, hipMemcpyHostToDevice));
    IB_HIP(hipMemcpy(w->ib_xyz, xyz.data(), nib * 8, hipMemcpyHostToDevice));
    IB_HIP(hipMemcpy(w->ib_meta, meta.data(), nib * 16, hipMemcpyHostToDevice));
    IB_HIP(hipMemcpy(w->ib_sigma, sig.data(), nib * 8, hipMemcpyHostToDevice));
  }
  // every point of this table has a support wider than the LDS-tiled patch takes, so no
  // dense-range records are made (empty ranges keep the state set-up uniform)
  if ((s = dalloc_t(&w->dense_first, std::max<int64_t>(nib, 1))) || (s = dalloc_t(&w->dense_count, std::max<int64_t>(nib, 1))) ||
      (s = dalloc_t(&w->dense_off, std::max<int64_t>(nib, 1))) || (s = dalloc_t(&w->dense32, 1)) || (s = dalloc_t(&w->dense64, 1)))
    return s;
  IB_HIP(hipMemsetAsync(w->dense_first, 0, std::max<int64_t>(nib, 1) * 4, st));
  IB_HIP(hipMemsetAsync(w->dense_count, 0, std::max<int64_t>(nib, 1) * 4, st));
  IB_HIP(hipMemsetAsync(w->dense_off, 0, std::max<int64_t>(nib, 1) * 4, st));
  IB_HIP(hipStreamSynchronize(st));
  w->dense_words = 0;
  w->stats.dense_weights = 0;
  return IB_OK;
}

}  // namespace ib
