// First-order (pressure-velocity) form on a staggered grid with its immersed boundary.
//
// Paper: "Extension to Multiple Fields and the 1st-Order Acoustic Wave Equation" and
// "The Particle Velocity Free-Surface".  p sits on the nodes, v_n at node + e_n / 2.
// Two families of modified operators:
//   gradient  d/dx_n p at v_n nodes whose staggered stencil reaches an exterior p node:
//             p is extrapolated about the v_n node (pressure hierarchy, eta_p);
//   divergence  div v at p nodes whose stencils reach exterior v nodes: all components
//             are extrapolated jointly about the p node, the divergence hierarchy rows
//             spanning every component block (eta_v, zero in the paper).
// The same boundary points (those of the p nodes) serve every field.
// Time stepping (signs as printed, rho = 1):
//   v^{n+1/2} = [(1 - s) v^{n-1/2} + (dt/h) D+ p^n] / (1 + s)
//   p^{n+1}   = [(1 - s) p^n + (dt c^2/h) D- . v^{n+1/2} + dt f^n] / (1 + s)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "ib_internal.h"
#include "step.h"
#include "surface.h"
#include "io.h"
#include "wave.h"

namespace ib {

// bit0 of the v_axis node classes: the node (position node + e_axis / 2) lies strictly on
// the physical side of the surface.
__global__ void k_classify_v(SurfView sv, uint8_t *cls, int nx, int ny, int nz, int axis, double sgn) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t N = (int64_t)nx * ny * nz;
  if (i >= N) return;
  const int x = (int)(i % nx);
  const int64_t r = i / nx;
  const int y = (int)(r % ny), z = (int)(r / ny);
  double H;
  double zz = z;
  if (axis == 2) {
    H = sv.Hs[(size_t)y * nx + x];
    zz = z + 0.5;
  } else {
    double g[2], hh[3];
    surf_eval(sv, x + (axis == 0 ? 0.5 : 0.0), y + (axis == 1 ? 0.5 : 0.0), H, g, hh);
  }
  cls[i] = (sgn * (zz - H) > 0.0) ? 1 : 0;
}

// bit1: exclusion of v nodes with a boundary point strictly inside their eta box
__global__ void k_exclude_v(const double *bp, int64_t nb, int nx, int ny, int nz, int lat, int axis, double eta,
                            uint8_t *cls) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nb || eta <= 0.0) return;
  double p[3] = {bp[j * 8 + 3], bp[j * 8 + 4], bp[j * 8 + 5]};
  p[axis] -= 0.5;   // position relative to the v node grid
  int lo[3], hi[3];
  for (int n = 0; n < 3; ++n) {
    lo[n] = (int)floor(p[n] - eta) + 1;
    hi[n] = (int)ceil(p[n] + eta) - 1;
  }
  if (lat == 1) lo[1] = hi[1] = 0;
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

// family flags: gradient (rows: v_axis nodes, reads p at +(m - 1/2), m = -H+1..H) or
// divergence (rows: p nodes, reads v_n at +(m + 1/2), m = -H..H-1, any n)
__global__ void k_flags_pv(const uint8_t *rowcls, const uint8_t *c0, const uint8_t *c1, const uint8_t *c2, int nx,
                           int ny, int nz, int half, int family, int axis, uint8_t *flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t N = (int64_t)nx * ny * nz;
  if (i >= N) return;
  flag[i] = 0;
  if (!(rowcls[i] & 1)) return;
  const int x = (int)(i % nx);
  const int64_t r = i / nx;
  const int y = (int)(r % ny), z = (int)(r / ny);
  auto ext = [&](const uint8_t *c, int n, int m) {
    int xx = x, yy = y, zz = z;
    if (n == 0) xx = wrapi(x + m, nx);
    if (n == 1) yy = wrapi(y + m, ny);
    if (n == 2) zz = z + m;
    if (zz < 0 || zz >= nz) return false;
    return !(c[((int64_t)zz * ny + yy) * nx + xx] & 1);
  };
  bool hit = false;
  if (family == 1) {
    for (int m = -half + 1; m <= half && !hit; ++m) hit = ext(c0, axis, m);
  } else {
    const uint8_t *cs[3] = {c0, c1, c2};
    for (int n = 0; n < 3 && !hit; ++n) {
      if (!cs[n]) continue;
      for (int m = -half; m <= half - 1 && !hit; ++m) hit = ext(cs[n], n, m);
    }
  }
  flag[i] = hit ? 1 : 0;
}

static std::vector<int64_t> compact(const uint8_t *flag_dev, int64_t N, hipStream_t st, ib_status &s) {
  std::vector<uint8_t> h(N);
  std::vector<int64_t> out;
  hipError_t e = hipMemcpyAsync(h.data(), flag_dev, N, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    s = hip_fail(e, "flag copy", __FILE__, __LINE__);
    return out;
  }
  for (int64_t i = 0; i < N; ++i)
    if (h[i]) out.push_back(i);
  s = IB_OK;
  return out;
}

// the velocity axes of a grid: (x, z) in 2D, (x, y, z) in 3D
static int vaxis(int ndim, int n) { return (ndim == 2 && n == 1) ? 2 : n; }

ib_status pv_build(ib_weights *w, const int64_t *col_off_dev, hipStream_t st) {
  const int ndim = w->ndim, lat = ndim - 1, nv = ndim;
  const int T = 256;
  const int half = w->M / 2;
  ib_status s;
  SurfView sv{w->Hs, (int)w->nx, (int)w->ny, lat};
  for (int n = 0; n < nv; ++n) {
    if ((s = dalloc_t(&w->vcls[n], w->N))) return s;
    hipLaunchKernelGGL(k_classify_v, dim3((unsigned)((w->N + T - 1) / T)), dim3(T), 0, st, sv, w->vcls[n], (int)w->nx,
                       (int)w->ny, (int)w->nz, vaxis(ndim, n), w->prm.physical_below ? 1.0 : -1.0);
    if (w->nb > 0 && w->prm.eta_v > 0.0)
      hipLaunchKernelGGL(k_exclude_v, dim3((unsigned)((w->nb + T - 1) / T)), dim3(T), 0, st, w->bp, w->nb, (int)w->nx,
                         (int)w->ny, (int)w->nz, lat, vaxis(ndim, n), w->prm.eta_v, w->vcls[n]);
  }
  IB_HIP(hipGetLastError());
  uint8_t *flag = nullptr;
  if ((s = dalloc_t(&flag, w->N))) return s;
  w->pv_row_fam.clear();
  w->pv_row_node.clear();
  w->pv_row_start.assign(1, 0);
  w->pv_ent_field.clear();
  w->pv_ent_node.clear();
  w->pv_ent_w.clear();
  auto emit = [&](int fam, const FamilySpec &F, const std::vector<FamilyPoint> &res) {
    for (size_t i = 0; i < res.size(); ++i) {
      const int64_t g = F.anchors[i];
      const int64_t x = g % w->nx, y = (g / w->nx) % w->ny, z = g / (w->nx * w->ny);
      w->pv_row_fam.push_back(fam);
      w->pv_row_node.push_back(g);
      for (size_t k = 0; k < res[i].w.size(); ++k) {
        const uint32_t v = (uint32_t)res[i].off[k];
        const int dx = (int8_t)(v & 255), dy = (int8_t)((v >> 8) & 255), dz = (int8_t)((v >> 16) & 255);
        const int64_t xx = ((x + dx) % w->nx + w->nx) % w->nx, yy = ((y + dy) % w->ny + w->ny) % w->ny;
        w->pv_ent_field.push_back(fam < nv ? -1 : res[i].field[k]);
        w->pv_ent_node.push_back((z + dz) * w->nx * w->ny + yy * w->nx + xx);
        w->pv_ent_w.push_back(res[i].w[k]);
      }
      w->pv_row_start.push_back((int64_t)w->pv_ent_w.size());
      w->stats.radius_hist[std::min(res[i].k, 7)]++;
      w->stats.order_hist[std::min(res[i].Mb, 16)]++;
    }
  };
  // gradient family, one per velocity component
  for (int n = 0; n < nv; ++n) {
    const int ax = vaxis(ndim, n);
    hipLaunchKernelGGL(k_flags_pv, dim3((unsigned)((w->N + T - 1) / T)), dim3(T), 0, st, w->vcls[n], w->node_class,
                       (const uint8_t *)nullptr, (const uint8_t *)nullptr, (int)w->nx, (int)w->ny, (int)w->nz, half, 1,
                       ax, flag);
    FamilySpec F;
    F.family = 1;
    F.gaxis = ax;
    F.nfields = 1;
    F.nblocks = 1;
    F.fcls[0] = w->node_class;
    F.x0off[ax] = 0.5;
    F.xcls[0] = w->node_class;
    F.anchors = compact(flag, w->N, st, s);
    if (s) return s;
    std::vector<FamilyPoint> res;
    if ((s = solve_family(w, F, col_off_dev, st, res))) return s;
    w->pv_stats[n] = (int64_t)res.size();
    emit(n, F, res);
  }
  // divergence family
  {
    const uint8_t *vc[3] = {nullptr, nullptr, nullptr};
    for (int n = 0; n < nv; ++n) vc[vaxis(ndim, n)] = w->vcls[n];
    hipLaunchKernelGGL(k_flags_pv, dim3((unsigned)((w->N + T - 1) / T)), dim3(T), 0, st, w->node_class, vc[0], vc[1],
                       vc[2], (int)w->nx, (int)w->ny, (int)w->nz, half, 2, 0, flag);
    FamilySpec F;
    F.family = 2;
    F.nfields = nv;
    F.nblocks = nv;
    for (int n = 0; n < nv; ++n) {
      const int ax = vaxis(ndim, n);
      F.fcls[n] = w->vcls[n];
      F.foff[n][ax] = 0.5;
      F.fblock[n] = n;
      F.baxis[n] = ax;
      F.xcls[n] = w->vcls[n];
    }
    F.anchors = compact(flag, w->N, st, s);
    if (s) return s;
    std::vector<FamilyPoint> res;
    if ((s = solve_family(w, F, col_off_dev, st, res))) return s;
    w->pv_stats[3] = (int64_t)res.size();
    emit(nv, F, res);
  }
  dfree(flag);
  w->nib = (int64_t)w->pv_row_fam.size();
  w->sumw = (int64_t)w->pv_ent_w.size();
  w->stats.n_ib = w->nib;
  w->stats.sum_nw = w->sumw;
  return IB_OK;
}

// ---- stepping ------------------------------------------------------------------------
template <typename T, int H>
__global__ void k_pv_velocity(T *__restrict__ v, const T *__restrict__ p, const T *__restrict__ kv,
                              const T *__restrict__ sx, const T *__restrict__ sy, const T *__restrict__ sz,
                              StaggerW<T> W, int nx, int ny, int nz, int64_t pitch, int64_t vol, int nv, int ndim,
                              int nshots) {
  const int64_t per = (int64_t)nx * ny * nz;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= per * nv * nshots) return;
  const int shot = (int)(g / (per * nv));
  int64_t rem = g % (per * nv);
  const int n = (int)(rem / per);
  int64_t i = rem % per;
  const int x = (int)(i % nx);
  i /= nx;
  const int y = (int)(i % ny), z = (int)(i / ny);
  const int ax = (ndim == 2 && n == 1) ? 2 : n;
  const int64_t plane = pitch * ny;
  const size_t c = (size_t)z * plane + (size_t)y * pitch + x;
  const T *pp = p + (size_t)shot * vol;
  T d = T(0);
#pragma unroll
  for (int m = -H + 1; m <= H; ++m) {
    int xx = x, yy = y, zz = z;
    if (ax == 0) xx = wrapi(x + m, nx);
    if (ax == 1) yy = wrapi(y + m, ny);
    if (ax == 2) zz = z + m;
    if (zz < 0 || zz >= nz) continue;
    d += W.w[m + H - 1] * pp[(size_t)zz * plane + (size_t)yy * pitch + xx];
  }
  const T s = sx[x] + sy[y] + sz[z];
  T *vv = v + ((size_t)shot * nv + n) * vol;
  vv[c] = ((T(1) - s) * vv[c] + kv[(size_t)n * vol + c] * d) / (T(1) + s);
}

template <typename T, int H>
__global__ void k_pv_pressure(T *__restrict__ p, const T *__restrict__ v, const T *__restrict__ kp,
                              const T *__restrict__ sx, const T *__restrict__ sy, const T *__restrict__ sz,
                              StaggerW<T> W, int nx, int ny, int nz, int64_t pitch, int64_t vol, int nv, int ndim,
                              int nshots) {
  const int64_t per = (int64_t)nx * ny * nz;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= per * nshots) return;
  const int shot = (int)(g / per);
  int64_t i = g % per;
  const int x = (int)(i % nx);
  i /= nx;
  const int y = (int)(i % ny), z = (int)(i / ny);
  const int64_t plane = pitch * ny;
  const size_t c = (size_t)z * plane + (size_t)y * pitch + x;
  T div = T(0);
  for (int n = 0; n < nv; ++n) {
    const int ax = (ndim == 2 && n == 1) ? 2 : n;
    const T *vv = v + ((size_t)shot * nv + n) * vol;
#pragma unroll
    for (int m = -H; m <= H - 1; ++m) {
      int xx = x, yy = y, zz = z;
      if (ax == 0) xx = wrapi(x + m, nx);
      if (ax == 1) yy = wrapi(y + m, ny);
      if (ax == 2) zz = z + m;
      if (zz < 0 || zz >= nz) continue;
      div += W.w[m + H] * vv[(size_t)zz * plane + (size_t)yy * pitch + xx];
    }
  }
  const T s = sx[x] + sy[y] + sz[z];
  T *q = p + (size_t)shot * vol;
  q[c] = ((T(1) - s) * q[c] + kp[c] * div) / (T(1) + s);
}

// 3D forms of the two updates: one thread per (x, y) column of a 64 x 4 tile marching down a
// chunk of zc planes.  The depth stencil comes from a register queue along z; the lateral
// stencils read neighbouring columns, which the tile's wavefronts share through the caches.
// The sums run in the same order as the one-node-per-thread kernels above.
template <typename T, int H>
__launch_bounds__(256)
__global__ void k_pv_velocity3d(T *__restrict__ v, const T *__restrict__ p, const uint8_t *__restrict__ c0,
                                const uint8_t *__restrict__ c1, const uint8_t *__restrict__ c2, T fv,
                                const T *__restrict__ sx, const T *__restrict__ sy, const T *__restrict__ sz,
                                StaggerW<T> W, int nx, int ny, int nz, int64_t pitch, int64_t vol, int zc,
                                const int2 *__restrict__ zr) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int nzc = (nz + zc - 1) / zc;
  const int shot = blockIdx.z / nzc;
  // the block's nzc chunks split evenly the planes that hold interior nodes of its columns
  // (the others hold zeros that stay zero)
  const int2 r = zr[blockIdx.y * gridDim.x + blockIdx.x];
  const int zcs = (r.y - r.x + nzc - 1) / nzc;
  const int z0 = r.x + (blockIdx.z - shot * nzc) * zcs;
  if (x >= nx || y >= ny) return;
  const int z1 = min(z0 + zcs, r.y);
  if (z0 >= z1) return;
  const int64_t plane = pitch * ny;
  const T *pp = p + (size_t)shot * vol;
  int xo[2 * H], yo[2 * H];
#pragma unroll
  for (int k = 0; k < 2 * H; ++k) {
    xo[k] = wrapi(x + k - H + 1, nx);
    yo[k] = wrapi(y + k - H + 1, ny) * (int)pitch;
  }
  T q[2 * H];   // p at z + k - H + 1
#pragma unroll
  for (int k = 0; k < 2 * H; ++k) {
    const int zz = z0 + k - H + 1;
    q[k] = (zz >= 0 && zz < nz) ? pp[(size_t)zz * plane + (size_t)y * pitch + x] : T(0);
  }
  const T sxy = sx[x] + sy[y];
  T *v0 = v + (size_t)shot * 3 * vol, *v1 = v0 + vol, *v2 = v1 + vol;
  for (int z = z0; z < z1; ++z) {
    const T *row = pp + (size_t)z * plane;
    const size_t c = (size_t)z * plane + (size_t)y * pitch + x;
    const size_t cu = ((size_t)z * ny + y) * nx + x;   // class arrays are unpadded
    // dt / h at interior v_n nodes, 0 elsewhere (the coefficient the 2D kernels read)
    const T k0 = (c0[cu] & 1) ? fv : T(0), k1 = (c1[cu] & 1) ? fv : T(0), k2 = (c2[cu] & 1) ? fv : T(0);
    T dx = T(0), dy = T(0), dz = T(0);
#pragma unroll
    for (int k = 0; k < 2 * H; ++k) dx += W.w[k] * row[(size_t)y * pitch + xo[k]];
#pragma unroll
    for (int k = 0; k < 2 * H; ++k) dy += W.w[k] * row[(size_t)yo[k] + x];
#pragma unroll
    for (int k = 0; k < 2 * H; ++k) dz += W.w[k] * q[k];
    const T s = sxy + sz[z];
    v0[c] = ((T(1) - s) * v0[c] + k0 * dx) / (T(1) + s);
    v1[c] = ((T(1) - s) * v1[c] + k1 * dy) / (T(1) + s);
    v2[c] = ((T(1) - s) * v2[c] + k2 * dz) / (T(1) + s);
#pragma unroll
    for (int k = 0; k < 2 * H - 1; ++k) q[k] = q[k + 1];
    const int zn = z + H + 1;
    q[2 * H - 1] = (zn < nz) ? pp[(size_t)zn * plane + (size_t)y * pitch + x] : T(0);
  }
}

template <typename T, int H>
__launch_bounds__(256)
__global__ void k_pv_pressure3d(T *__restrict__ p, const T *__restrict__ v, const T *__restrict__ kp,
                                const T *__restrict__ sx, const T *__restrict__ sy, const T *__restrict__ sz,
                                StaggerW<T> W, int nx, int ny, int nz, int64_t pitch, int64_t vol, int zc,
                                const int2 *__restrict__ zr) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int nzc = (nz + zc - 1) / zc;
  const int shot = blockIdx.z / nzc;
  // the block's nzc chunks split evenly the planes that hold interior nodes of its columns
  // (the others hold zeros that stay zero)
  const int2 r = zr[blockIdx.y * gridDim.x + blockIdx.x];
  const int zcs = (r.y - r.x + nzc - 1) / nzc;
  const int z0 = r.x + (blockIdx.z - shot * nzc) * zcs;
  if (x >= nx || y >= ny) return;
  const int z1 = min(z0 + zcs, r.y);
  if (z0 >= z1) return;
  const int64_t plane = pitch * ny;
  const T *v0 = v + (size_t)shot * 3 * vol, *v1 = v0 + vol, *v2 = v1 + vol;
  int xo[2 * H], yo[2 * H];
#pragma unroll
  for (int k = 0; k < 2 * H; ++k) {
    xo[k] = wrapi(x + k - H, nx);
    yo[k] = wrapi(y + k - H, ny) * (int)pitch;
  }
  T q[2 * H];   // v_z at z + k - H
#pragma unroll
  for (int k = 0; k < 2 * H; ++k) {
    const int zz = z0 + k - H;
    q[k] = (zz >= 0 && zz < nz) ? v2[(size_t)zz * plane + (size_t)y * pitch + x] : T(0);
  }
  const T sxy = sx[x] + sy[y];
  T *pp = p + (size_t)shot * vol;
  for (int z = z0; z < z1; ++z) {
    const size_t rz = (size_t)z * plane;
    const size_t c = rz + (size_t)y * pitch + x;
    T div = T(0);
#pragma unroll
    for (int k = 0; k < 2 * H; ++k) div += W.w[k] * v0[rz + (size_t)y * pitch + xo[k]];
#pragma unroll
    for (int k = 0; k < 2 * H; ++k) div += W.w[k] * v1[rz + (size_t)yo[k] + x];
#pragma unroll
    for (int k = 0; k < 2 * H; ++k) div += W.w[k] * q[k];
    const T s = sxy + sz[z];
    // p and its coefficient are streamed once: non-temporal (measured faster here; the
    // velocity kernel measured slower with the same hints)
    __builtin_nontemporal_store(
        ((T(1) - s) * __builtin_nontemporal_load(&pp[c]) + __builtin_nontemporal_load(&kp[c]) * div) / (T(1) + s),
        &pp[c]);
#pragma unroll
    for (int k = 0; k < 2 * H - 1; ++k) q[k] = q[k + 1];
    const int zn = z + H;
    q[2 * H - 1] = (zn < nz) ? v2[(size_t)zn * plane + (size_t)y * pitch + x] : T(0);
  }
}

// modified rows: dst[row] += scale[row] * sum_k w_k src[k].  A group of L lanes (8 or 16)
// takes one modified row: its lanes read the row's entries together, two entries per lane in
// flight, and the partial sums are combined by DPP inside the group; shots loop inside.
template <typename T, int L>
__launch_bounds__(256)
__global__ void k_pv_rows(T *__restrict__ dst, int64_t dst_shot_stride, const T *__restrict__ src,
                          int64_t src_shot_stride, const int64_t *__restrict__ rnode, const T *__restrict__ rscale,
                          const int64_t *__restrict__ rstart, const uint32_t *__restrict__ enode,
                          const T *__restrict__ ew, int64_t nrows, int nshots, PatchIo<T> io, T *pf,
                          int64_t pvol) {
  // the io workgroups first (sampling from, or injection into, the pressure field pf)
  const int blk = (int)blockIdx.x, nsp = io.nsb + io.ninj;
  if (blk < io.nsb) {
    sample_block(pf, io, blk, pvol);
    finish_io(io);
    return;
  }
  if (blk < nsp) {
    inject_sources(pf, (T *)nullptr, io.sidx, io.sw, nshots, pvol, io.wavelet, io.wstride, io.tcount[0]);
    finish_io(io);
    return;
  }
  const int sub = threadIdx.x & (L - 1);
  const int64_t r = (int64_t)(blk - nsp) * (blockDim.x / L) + threadIdx.x / L;
  const bool live = r < nrows;
  // rows stay complete (no early return) so that the DPP exchanges see all lanes
  const int64_t a = live ? rstart[r] : 0, b = live ? rstart[r + 1] : 0;
  for (int s = 0; s < nshots; ++s) {
    const T *ss = src + (size_t)s * src_shot_stride;
    T acc = T(0), acc1 = T(0);
    int64_t k = a + sub;
    for (; k + L < b; k += 2 * L) {
      const uint32_t e0 = enode[k], e1 = enode[k + L];
      const T w0 = ew[k], w1 = ew[k + L];
      const T p0 = ss[e0], p1 = ss[e1];
      acc += w0 * p0;
      acc1 += w1 * p1;
    }
    if (k < b) acc += ew[k] * ss[enode[k]];
    acc = (L == 16) ? row_sum16(acc + acc1) : row_sum8(acc + acc1);
    if (live && sub == 0) dst[(size_t)s * dst_shot_stride + rnode[r]] += rscale[r] * acc;
  }
}

template <typename T>
static StaggerW<T> stagger_weights(int M) {
  double w[kMaxOrder];
  staggered_first_derivative_weights(M, w);
  StaggerW<T> W{};
  for (int k = 0; k < M; ++k) W.w[k] = (T)w[k];
  return W;
}

template <typename T, int H>
static void pv_step_h(const PVArgs &a, hipStream_t st) {
  const int64_t per = (int64_t)a.nx * a.ny * a.nz;
  const StaggerW<T> W = stagger_weights<T>(a.M);
  dim3 b(256);
  dim3 gv((unsigned)((per * a.nv * a.nshots + 255) / 256)), gp((unsigned)((per * a.nshots + 255) / 256));
  const int zc = 32;
  const dim3 g3((unsigned)((a.nx + 63) / 64), (unsigned)((a.ny + 3) / 4),
                (unsigned)(((a.nz + zc - 1) / zc) * a.nshots));
  if (a.ndim == 3 && a.zr4)
    hipLaunchKernelGGL((k_pv_velocity3d<T, H>), g3, b, 0, st, (T *)a.v, (const T *)a.p, a.vcls[0], a.vcls[1],
                       a.vcls[2], (T)a.fv, (const T *)a.sx, (const T *)a.sy, (const T *)a.sz, W, a.nx, a.ny, a.nz,
                       a.pitch, a.vol, zc, a.zr4);
  else
    hipLaunchKernelGGL((k_pv_velocity<T, H>), gv, b, 0, st, (T *)a.v, (const T *)a.p, (const T *)a.kv,
                       (const T *)a.sx, (const T *)a.sy, (const T *)a.sz, W, a.nx, a.ny, a.nz, a.pitch, a.vol, a.nv,
                       a.ndim, a.nshots);
  // the sources and receivers (io_merge): sampling for the step before in the gradient
  // rows, which read p; injection and the counter's advance in the divergence rows
  PatchIo<T> gio{}, dio{};
  if (a.io_merge) {
    if (a.sample_prev && a.nrec > 0 && a.traces) {
      gio.ridx = a.ridx;
      gio.rw = (const T *)a.rw;
      gio.nrec = a.nrec;
      gio.nrs = (int64_t)a.nrec * a.nshots;
      gio.nsb = (int)std::min<int64_t>((gio.nrs + 255) / 256, kMaxSampleBlocks);
      gio.traces = (T *)a.traces;
      gio.nsteps = a.nsteps;
      gio.tcount = a.tcount;
    }
    dio.sidx = a.sidx;
    dio.sw = (const T *)a.sw;
    dio.wavelet = (const T *)a.wavelet;
    dio.wstride = a.wstride;
    dio.ninj = 1;
    dio.tcount = a.tcount;
    dio.advance = 1;
  }
  if (a.nrows_g > 0) {
    if (a.g_lanes == 8)
      hipLaunchKernelGGL((k_pv_rows<T, 8>), dim3((unsigned)((a.nrows_g + 31) / 32 + gio.nsb)), b, 0, st, (T *)a.v,
                         (int64_t)a.nv * a.vol, (const T *)a.p, a.vol, a.g_node, (const T *)a.g_scale, a.g_start,
                         a.g_enode, (const T *)a.g_w, a.nrows_g, a.nshots, gio, (T *)a.p, a.vol);
    else
      hipLaunchKernelGGL((k_pv_rows<T, 16>), dim3((unsigned)((a.nrows_g + 15) / 16 + gio.nsb)), b, 0, st, (T *)a.v,
                         (int64_t)a.nv * a.vol, (const T *)a.p, a.vol, a.g_node, (const T *)a.g_scale, a.g_start,
                         a.g_enode, (const T *)a.g_w, a.nrows_g, a.nshots, gio, (T *)a.p, a.vol);
  }
  if (a.ndim == 3 && a.zr4)
    hipLaunchKernelGGL((k_pv_pressure3d<T, H>), g3, b, 0, st, (T *)a.p, (const T *)a.v, (const T *)a.kp,
                       (const T *)a.sx, (const T *)a.sy, (const T *)a.sz, W, a.nx, a.ny, a.nz, a.pitch, a.vol, zc,
                       a.zr4);
  else
    hipLaunchKernelGGL((k_pv_pressure<T, H>), gp, b, 0, st, (T *)a.p, (const T *)a.v, (const T *)a.kp,
                       (const T *)a.sx, (const T *)a.sy, (const T *)a.sz, W, a.nx, a.ny, a.nz, a.pitch, a.vol, a.nv,
                       a.ndim, a.nshots);
  if (a.nrows_d > 0) {
    if (a.d_lanes == 8)
      hipLaunchKernelGGL((k_pv_rows<T, 8>), dim3((unsigned)((a.nrows_d + 31) / 32 + dio.ninj)), b, 0, st, (T *)a.p,
                         a.vol, (const T *)a.v, (int64_t)a.nv * a.vol, a.d_node, (const T *)a.d_scale, a.d_start,
                         a.d_enode, (const T *)a.d_w, a.nrows_d, a.nshots, dio, (T *)a.p, a.vol);
    else
      hipLaunchKernelGGL((k_pv_rows<T, 16>), dim3((unsigned)((a.nrows_d + 15) / 16 + dio.ninj)), b, 0, st, (T *)a.p,
                         a.vol, (const T *)a.v, (int64_t)a.nv * a.vol, a.d_node, (const T *)a.d_scale, a.d_start,
                         a.d_enode, (const T *)a.d_w, a.nrows_d, a.nshots, dio, (T *)a.p, a.vol);
  }
}

template <typename T>
static void pv_step_t(const PVArgs &a, hipStream_t st) {
  switch (a.M / 2) {
    case 1: pv_step_h<T, 1>(a, st); break;
    case 2: pv_step_h<T, 2>(a, st); break;
    case 3: pv_step_h<T, 3>(a, st); break;
    default: pv_step_h<T, 4>(a, st); break;
  }
}

void enqueue_pv_step(const PVArgs &a, hipStream_t st) {
  if (a.prec == IB_F32)
    pv_step_t<float>(a, st);
  else
    pv_step_t<double>(a, st);
}

}  // namespace ib
