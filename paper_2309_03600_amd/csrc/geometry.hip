// Surface geometry on the GPU (FP64): node classes, boundary points, eta exclusion,
// immersed-boundary points.
//
// The surface is the heightfield z = H(x[, y]) through the column samples, continued by
// the periodic Catmull-Rom cubic (tensor product in 3D).  Boundary points follow the
// paper's rule (section "Approximating Boundary Conditions"): the closest surface point
// of a node - where the surface normal through the node meets the surface - kept when
// it lies in the node's half-open one-cell box.  The closest point is located by a
// coarse search over lateral offsets -1..1 in steps of 1/8 followed by Newton's method
// on |(xi, H(xi)) - x|^2 with step halving.  Interior nodes with a boundary point
// strictly inside their box of half-width eta are excluded from extrapolation data.
#include <hip/hip_runtime.h>

#include "ib_internal.h"
#include "surface.h"

namespace ib {

__device__ __forceinline__ double objective(const SurfView &s, double u, double v, double xu, double xv,
                                            double z) {
  double H, g[2], hh[3];
  surf_eval(s, u, v, H, g, hh);
  double du = u - xu, dv = (s.lat == 2) ? v - xv : 0.0, dz = H - z;
  return du * du + dv * dv + dz * dz;
}

// Closest surface point of node (xu, xv, z); returns (u, v, H(u, v)).
__device__ void foot_point(const SurfView &s, double xu, double xv, double z, double out[3]) {
  const int steps = 8;
  double best = INFINITY, bu = xu, bv = xv;
  int nb = (s.lat == 2) ? 2 * steps + 1 : 1;
  for (int a = 0; a <= 2 * steps; ++a) {
    double ou = -1.0 + (double)a / steps;
    for (int b = 0; b < nb; ++b) {
      double ov = (s.lat == 2) ? -1.0 + (double)b / steps : 0.0;
      double F = objective(s, xu + ou, xv + ov, xu, xv, z);
      if (F < best) {
        best = F;
        bu = xu + ou;
        bv = xv + ov;
      }
    }
  }
  double u = bu, v = bv;
  for (int it = 0; it < 20; ++it) {
    double H, g[2], hh[3];
    surf_eval(s, u, v, H, g, hh);
    double r = H - z;
    double su, sv;
    if (s.lat == 1) {
      double grad = 2.0 * (u - xu) + 2.0 * r * g[0];
      double hs = 2.0 + 2.0 * g[0] * g[0] + 2.0 * r * hh[0];
      su = (hs > 0.0) ? -grad / hs : -0.5 * grad;
      sv = 0.0;
    } else {
      double gu = 2.0 * (u - xu) + 2.0 * r * g[0];
      double gv = 2.0 * (v - xv) + 2.0 * r * g[1];
      double a = 2.0 + 2.0 * g[0] * g[0] + 2.0 * r * hh[0];
      double b = 2.0 * g[0] * g[1] + 2.0 * r * hh[1];
      double d = 2.0 + 2.0 * g[1] * g[1] + 2.0 * r * hh[2];
      double det = a * d - b * b;
      if (a > 0.0 && det > 0.0) {
        su = -(d * gu - b * gv) / det;
        sv = -(-b * gu + a * gv) / det;
      } else {
        su = -0.5 * gu;
        sv = -0.5 * gv;
      }
    }
    // halve only long steps: below 1e-6 the objective's change is under its rounding
    // error, and the Newton iteration converges quadratically on its own
    double F0 = objective(s, u, v, xu, xv, z);
    for (int hlv = 0; hlv < 30; ++hlv) {
      if (!(fmax(fabs(su), fabs(sv)) > 1e-6)) break;
      double F1 = objective(s, u + su, v + sv, xu, xv, z);
      if (!(F1 > F0)) break;
      su *= 0.5;
      sv *= 0.5;
    }
    u += su;
    v += sv;
    if (fmax(fabs(su), fabs(sv)) < 1e-13) break;
  }
  double H, g[2], hh[3];
  surf_eval(s, u, v, H, g, hh);
  out[0] = u;
  out[1] = v;
  out[2] = H;
}

__global__ void k_scale_heights(const double *H, double *Hs, int64_t n, double h) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) Hs[i] = H[i] / h;
}

// bit0: interior (strictly on the physical side; for a heightfield, the sign of z - H
// at the node's own column).
__global__ void k_classify(const double *Hs, uint8_t *cls, int nx, int ny, int nz, double sgn) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t N = (int64_t)nx * ny * nz;
  if (i >= N) return;
  int x = (int)(i % nx);
  int64_t r = i / nx;
  int y = (int)(r % ny);
  int z = (int)(r / ny);
  double H = Hs[(size_t)y * nx + x];
  cls[i] = (sgn * ((double)z - H) > 0.0) ? 1 : 0;
}

// Candidate depth range per column: within 1.5 cells of the surface's range over the
// coarse lateral window.
__global__ void k_column_range(SurfView s, int nz, int *k0, int *k1) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (int64_t)s.nx * s.ny) return;
  int x = (int)(c % s.nx), y = (int)(c / s.nx);
  double lo = INFINITY, hi = -INFINITY;
  int nb = (s.lat == 2) ? 17 : 1;
  for (int a = 0; a <= 16; ++a)
    for (int b = 0; b < nb; ++b) {
      double H, g[2], hh[3];
      surf_eval(s, x - 1.0 + a / 8.0, (s.lat == 2) ? y - 1.0 + b / 8.0 : 0.0, H, g, hh);
      lo = fmin(lo, H);
      hi = fmax(hi, H);
    }
  int a0 = (int)fmax(ceil(lo - 1.5), 0.0);
  int a1 = (int)fmin(floor(hi + 1.5), (double)(nz - 1));
  k0[c] = a0;
  k1[c] = a1;
}

// One thread per (column, candidate slot).  Pass 0 counts hosted boundary points per
// column; pass 1 writes them at the column's offset in column order.
__global__ void k_boundary_points(SurfView s, int nz, const int *k0, const int *k1, int maxc, int pass,
                                  int *count, const int64_t *offset, double *bp, double *bpn,
                                  uint8_t *cls) {
  int64_t c = (int64_t)blockIdx.x;
  int slot = threadIdx.x + blockIdx.y * blockDim.x;
  if (c >= (int64_t)s.nx * s.ny) return;
  int z = k0[c] + slot;
  if (slot >= maxc || z > k1[c]) return;
  int x = (int)(c % s.nx), y = (int)(c / s.nx);
  double f[3];
  foot_point(s, (double)x, (double)y, (double)z, f);
  double rx = f[0] - x, ry = (s.lat == 2) ? f[1] - y : 0.0, rz = f[2] - z;
  bool hosted = rx >= -0.5 && rx < 0.5 && ry >= -0.5 && ry < 0.5 && rz >= -0.5 && rz < 0.5;
  if (!hosted) return;
  // position of this point inside its column: hosted candidates below it in the column
  if (pass == 0) {
    atomicAdd(&count[c], 1);
    return;
  }
  int rank = 0;
  for (int zz = k0[c]; zz < z; ++zz) {
    double g[3];
    foot_point(s, (double)x, (double)y, (double)zz, g);
    double ax = g[0] - x, ay = (s.lat == 2) ? g[1] - y : 0.0, az = g[2] - zz;
    if (ax >= -0.5 && ax < 0.5 && ay >= -0.5 && ay < 0.5 && az >= -0.5 && az < 0.5) ++rank;
  }
  int64_t j = offset[c] + rank;
  double *o = bp + j * 8;
  o[0] = x;
  o[1] = (s.lat == 2) ? y : 0.0;
  o[2] = z;
  o[3] = f[0];
  o[4] = (s.lat == 2) ? f[1] : 0.0;
  o[5] = f[2];
  o[6] = 0.0;
  o[7] = 0.0;
  double H, g[2], hh[3];
  surf_eval(s, f[0], f[1], H, g, hh);
  double nx_ = -g[0], ny_ = (s.lat == 2) ? -g[1] : 0.0, nz_ = 1.0;
  double nn = sqrt(nx_ * nx_ + ny_ * ny_ + nz_ * nz_);
  bpn[j * 3 + 0] = nx_ / nn;
  bpn[j * 3 + 1] = ny_ / nn;
  bpn[j * 3 + 2] = nz_ / nn;
  int64_t node = ((int64_t)z * s.ny + y) * s.nx + x;
  cls[node] |= 8;
}

// bit1: interior node with a boundary point strictly inside its half-width-eta box.
__global__ void k_exclude(const double *bp, int64_t nb, int nx, int ny, int nz, int lat, double eta,
                          uint8_t *cls) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nb || eta <= 0.0) return;
  const double *p = bp + j * 8 + 3;
  int lo[3], hi[3];
  for (int n = 0; n < 3; ++n) {
    lo[n] = (int)floor(p[n] - eta) + 1;
    hi[n] = (int)ceil(p[n] + eta) - 1;
  }
  if (lat == 1) {
    lo[1] = 0;
    hi[1] = 0;
  }
  for (int gz = lo[2]; gz <= hi[2]; ++gz) {
    if (gz < 0 || gz >= nz || !(fabs(p[2] - gz) < eta)) continue;
    for (int gy = lo[1]; gy <= hi[1]; ++gy) {
      if (lat == 2 && !(fabs(p[1] - gy) < eta)) continue;
      for (int gx = lo[0]; gx <= hi[0]; ++gx) {
        if (!(fabs(p[0] - gx) < eta)) continue;
        int64_t node = ((int64_t)gz * ny + wrapi(gy, ny)) * nx + wrapi(gx, nx);
        if (cls[node] & 1) cls[node] |= 2;
      }
    }
  }
}

// bit2: interior node whose axis stencils (+-1..M/2) reach an exterior node inside the
// box (outside the box the field is zero padding, not an exterior to extrapolate).
__global__ void k_ib_flags(uint8_t *cls, int nx, int ny, int nz, int lat, int half, uint8_t *flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t N = (int64_t)nx * ny * nz;
  if (i >= N) return;
  flag[i] = 0;
  if (!(cls[i] & 1)) return;
  int x = (int)(i % nx);
  int64_t r = i / nx;
  int y = (int)(r % ny);
  int z = (int)(r / ny);
  bool ib = false;
  for (int k = 1; k <= half && !ib; ++k) {
    for (int sg = -1; sg <= 1; sg += 2) {
      int xx = wrapi(x + sg * k, nx);
      if (!(cls[((int64_t)z * ny + y) * nx + xx] & 1)) ib = true;
      if (lat == 2) {
        int yy = wrapi(y + sg * k, ny);
        if (!(cls[((int64_t)z * ny + yy) * nx + x] & 1)) ib = true;
      }
      int zz = z + sg * k;
      if (zz >= 0 && zz < nz && !(cls[((int64_t)zz * ny + y) * nx + x] & 1)) ib = true;
    }
  }
  if (ib) {
    cls[i] |= 4;
    flag[i] = 1;
  }
}

// ---- host drivers ------------------------------------------------------------------

ib_status geometry_build(ib_weights *w, const double *height_dev, hipStream_t st) {
  const int lat = w->ndim - 1;
  const int64_t ncol = w->nx * w->ny;
  IB_HIP(hipGetLastError());
  ib_status s;
  if ((s = dalloc_t(&w->Hs, ncol))) return s;
  if ((s = dalloc_t(&w->node_class, w->N))) return s;
  const int T = 256;
  hipLaunchKernelGGL(k_scale_heights, dim3((ncol + T - 1) / T), dim3(T), 0, st, height_dev, w->Hs, ncol,
                     w->h);
  hipLaunchKernelGGL(k_classify, dim3((w->N + T - 1) / T), dim3(T), 0, st, w->Hs, w->node_class, (int)w->nx,
                     (int)w->ny, (int)w->nz, w->prm.physical_below ? 1.0 : -1.0);
  IB_HIP(hipGetLastError());
  SurfView sv{w->Hs, (int)w->nx, (int)w->ny, lat};
  int *k0 = nullptr, *k1 = nullptr, *cnt = nullptr;
  int64_t *off = nullptr;
  if ((s = dalloc_t(&k0, ncol)) || (s = dalloc_t(&k1, ncol)) || (s = dalloc_t(&cnt, ncol)) ||
      (s = dalloc_t(&off, ncol))) {
    dfree(k0), dfree(k1), dfree(cnt), dfree(off);
    return s;
  }
  hipLaunchKernelGGL(k_column_range, dim3((ncol + T - 1) / T), dim3(T), 0, st, sv, (int)w->nz, k0, k1);
  std::vector<int> h0(ncol), h1(ncol);
  IB_HIP(hipMemcpyAsync(h0.data(), k0, ncol * sizeof(int), hipMemcpyDeviceToHost, st));
  IB_HIP(hipMemcpyAsync(h1.data(), k1, ncol * sizeof(int), hipMemcpyDeviceToHost, st));
  IB_HIP(hipStreamSynchronize(st));
  int maxc = 0;
  for (int64_t c = 0; c < ncol; ++c) maxc = std::max(maxc, h1[c] - h0[c] + 1);
  maxc = std::max(maxc, 1);
  IB_HIP(hipMemsetAsync(cnt, 0, ncol * sizeof(int), st));
  int bx = std::min(64, maxc);
  dim3 grid((unsigned)ncol, (unsigned)((maxc + bx - 1) / bx));
  hipLaunchKernelGGL(k_boundary_points, grid, dim3(bx), 0, st, sv, (int)w->nz, k0, k1, maxc, 0, cnt,
                     (const int64_t *)nullptr, (double *)nullptr, (double *)nullptr, w->node_class);
  IB_HIP(hipGetLastError());
  std::vector<int> hc(ncol);
  std::vector<int64_t> ho(ncol);
  IB_HIP(hipMemcpyAsync(hc.data(), cnt, ncol * sizeof(int), hipMemcpyDeviceToHost, st));
  IB_HIP(hipStreamSynchronize(st));
  int64_t nb = 0;
  for (int64_t c = 0; c < ncol; ++c) {
    ho[c] = nb;
    nb += hc[c];
  }
  w->nb = nb;
  IB_HIP(hipMemcpyAsync(off, ho.data(), ncol * sizeof(int64_t), hipMemcpyHostToDevice, st));
  if ((s = dalloc_t(&w->bp, nb * 8)) || (s = dalloc_t(&w->bp_normal, nb * 3))) return s;
  hipLaunchKernelGGL(k_boundary_points, grid, dim3(bx), 0, st, sv, (int)w->nz, k0, k1, maxc, 1, cnt, off,
                     w->bp, w->bp_normal, w->node_class);
  IB_HIP(hipGetLastError());
  if (nb > 0)
    hipLaunchKernelGGL(k_exclude, dim3((nb + T - 1) / T), dim3(T), 0, st, w->bp, nb, (int)w->nx, (int)w->ny,
                       (int)w->nz, lat, w->prm.eta, w->node_class);
  IB_HIP(hipGetLastError());
  IB_HIP(hipStreamSynchronize(st));
  dfree(k0), dfree(k1), dfree(cnt), dfree(off);
  return IB_OK;
}

ib_status ib_points_build(ib_weights *w, hipStream_t st) {
  const int T = 256;
  const int lat = w->ndim - 1;
  uint8_t *flag = nullptr;
  ib_status s;
  if ((s = dalloc_t(&flag, w->N))) return s;
  hipLaunchKernelGGL(k_ib_flags, dim3((w->N + T - 1) / T), dim3(T), 0, st, w->node_class, (int)w->nx,
                     (int)w->ny, (int)w->nz, lat, w->M / 2, flag);
  IB_HIP(hipGetLastError());
  // compaction in memory order on the host (a setup step; N bytes cross PCIe once)
  std::vector<uint8_t> hf(w->N);
  IB_HIP(hipMemcpyAsync(hf.data(), flag, w->N, hipMemcpyDeviceToHost, st));
  IB_HIP(hipStreamSynchronize(st));
  dfree(flag);
  std::vector<int64_t> nodes;
  for (int64_t i = 0; i < w->N; ++i)
    if (hf[i]) nodes.push_back(i);
  w->nib = (int64_t)nodes.size();
  if ((s = dalloc_t(&w->ib_node, std::max<int64_t>(w->nib, 1)))) return s;
  IB_HIP(hipMemcpyAsync(w->ib_node, nodes.data(), w->nib * sizeof(int64_t), hipMemcpyHostToDevice, st));
  IB_HIP(hipStreamSynchronize(st));
  return IB_OK;
}

}  // namespace ib
