// Time-stepping kernels of the second-order pressure form.
//
// One step (section "Application to the 2nd-Order Acoustic Wave Equation", with the
// damping layer as a separable addition):
//   p^{n+1} = [2 p^n - (1 - s) p^{n-1} + K (L p^n) + dt^2 f^n] / (1 + s)
// split into
//   k_interior*  standard cross stencil at every node (exterior nodes have K = 0 and
//                stay zero), written over p^{n-1};
//   k_patch      at every IB point adds K/(1+s) * sum_j y_j p^n_j, the extrapolation
//                part of the modified Laplacian (the exterior values the interior
//                stencil reads are zero, so the standard part is already complete);
//   k_inject     point sources (also advances the device step counter);
//   k_sample     receivers (k_io_small does both in one launch for few receivers).
//
// Increment form (FP32 states): the state keeps d^n = p^n - p^{n-1} in place of p^{n-1},
//   d^{n+1} = [(1 - s) d^n + K (L p^n) + dt^2 f^n] / (1 + s),   p^{n+1} = p^n + d^{n+1},
// the same recurrence rearranged.  Rounding p^{n+1} to the storage precision then perturbs
// the field but not its time difference, so round-off does not build up as a velocity
// error that the leapfrog carries along; every term added after the interior kernel (IB
// patch, sources, boundary values) goes into both d^{n+1} and p^{n+1}.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "ib_internal.h"
#include "step.h"
#include "io.h"
#include "wave.h"

namespace ib {


template <typename T>
struct StencilW {
  T w[kMaxOrder / 2 + 1];   // w[0] centre, w[k] offset +-k
};


// The increment form's Laplacian: sum_k w_k ((p_{-k} - p_0) + (p_{+k} - p_0)) over the axes,
// equal to the centred stencil because its weights annihilate constants.  The centre term
// w_0 p_0 is several times larger than the Laplacian of a resolved wave and cancels
// against the neighbours; the differences are small (and exact when neighbours lie within
// a factor of two), so this order leaves a rounding error several times smaller.  get(k,
// side) returns the neighbour at offset k on side 0..5 (-x, +x, -y, +y, -z, +z).
template <int H, typename T, typename G>
__device__ __forceinline__ T lap_diff(const StencilW<T> &W, T c, G get) {
  T lap = T(0);
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    const T sk = ((get(k, 0) - c) + (get(k, 1) - c)) + ((get(k, 2) - c) + (get(k, 3) - c)) +
                 ((get(k, 4) - c) + (get(k, 5) - c));
    lap = fma(W.w[k], sk, lap);
  }
  return lap;
}

// d^{n+1} = [(1 - s) d^n + K lap] / (1 + s); outside the damping layer (s = 0) the division
// is by one and is skipped
template <typename T>
__device__ __forceinline__ T increment(T K, T lap, T d, T s) {
  if (s == T(0)) return fma(K, lap, d);
  return fma(K, lap, mul_rn(T(1) - s, d)) / (T(1) + s);
}

__device__ __forceinline__ int wrapk(int i, int n) {
  return i < 0 ? i + n : (i >= n ? i - n : i);
}

// XCD-aware block order: the hardware deals consecutive workgroups to the 8 XCDs in
// turn; remap so that each XCD walks a contiguous range of tiles (shared halos in its L2).
// ``nblk`` (the launched grid) must be a multiple of 8 so that the map is a permutation.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nblk) {
  int64_t per = (nblk + 7) / 8;
  return (b % 8) * per + b / 8;
}

// ---- buffer loads ---------------------------------------------------------------------
// A raw buffer resource over [base, base + bytes): a load at an offset out of that range
// returns 0 without a memory access, which makes conditional loads branch-free (all of a
// thread's loads are issued before the first result is needed) and skips the traffic of
// the nodes left out.
constexpr uint32_t kBufOff = 0x80000000u;   // an offset out of range (bytes < 2^31)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

// Stage p^n of SC shots over an LDS tile of LZ x LY x LX nodes (with PAD = 1 the last x of
// each row is padding) whose node (0, 0, 0) is grid node (gx0, gy0, gz0), laterally
// periodic: each of the NT threads issues all its loads, then writes them.  keep(lx, ly, lz)
// leaves a node out (zero) when false; nodes above or below the box are zero.  The caller
// checks that a shot's volume is under 2^31 bytes.
// (LDS rows RP apart and planes PL apart: RP = LX, PL = LX * LY is the dense layout; with ILV
// the SC shots of a node sit side by side, else shot c starts spstride values after shot 0)
template <typename T, int SC, int LX, int LY, int LZ, int NT, int PAD, typename Keep, int RP = LX, int PL = LX * LY,
          bool ILV = false>
__device__ __forceinline__ void stage_tile(T *sp, int spstride, const T *un, int64_t vol, int s0, int nshots, int gx0,
                                           int gy0, int gz0, int nx, int ny, int nz, int64_t pitch, Keep keep) {
  constexpr int N = LX * LY * LZ, NST = (N + NT - 1) / NT;
  // an opaque thread index keeps the address arithmetic in here: hoisted out of the
  // caller's loop over shot passes it would hold NST more registers for the whole kernel
  int tid = (int)threadIdx.x;
  __asm__ volatile("" : "+v"(tid));
  __amdgpu_buffer_rsrc_t r[SC];
#pragma unroll
  for (int c = 0; c < SC; ++c)
    r[c] = buf_rsrc(un + (size_t)(s0 + c) * vol, (s0 + c < nshots) ? (uint32_t)(vol * (int64_t)sizeof(T)) : 0u);
  T v[SC][NST];
#pragma unroll
  for (int j = 0; j < NST; ++j) {
    const int e = tid + j * NT;
    const int lx = e % LX, ly = (e / LX) % LY, lz = e / (LX * LY);
    const int gz = gz0 + lz;
    const bool in = e < N && (PAD == 0 || lx < LX - 1) && gz >= 0 && gz < nz && keep(lx, ly, lz);
    const int gx = wrapk(gx0 + lx, nx), gy = wrapk(gy0 + ly, ny);
    const uint32_t off = in ? (uint32_t)(((int64_t)gz * ny + gy) * pitch + gx) * (uint32_t)sizeof(T) : kBufOff;
#pragma unroll
    for (int c = 0; c < SC; ++c) v[c][j] = buf_load(r[c], off, T(0));
  }
#pragma unroll
  for (int j = 0; j < NST; ++j) {
    const int e = tid + j * NT;
    if (e < N) {
      const int lx = e % LX, ly = (e / LX) % LY, lz = e / (LX * LY);
#pragma unroll
      for (int c = 0; c < SC; ++c) {
        const int node = lz * PL + ly * RP + lx;
        sp[ILV ? node * SC + c : c * spstride + node] = v[c][j];
      }
    }
  }
}

// ---- 3D interior: xy tile in LDS, register queue along z ---------------------------
template <typename T, int H, int RY, bool DL>
__launch_bounds__(256)
__global__ void k_interior3d(const T *__restrict__ un, T *__restrict__ um, T *__restrict__ dd, const T *__restrict__ K,
                             const T *__restrict__ sx, const T *__restrict__ sy, const T *__restrict__ sz,
                             StencilW<T> W, StencilW<double> WD, int nx, int ny, int nz, int64_t pitch, int64_t vol,
                             int zchunk, int ntx, int nty, int nzc, int nshots) {
  constexpr int TX = 64, TY = 4 * RY, LX = TX + 2 * H, LY = TY + 2 * H;
  __shared__ T tile[LY][LX];
  const int64_t nblk = (int64_t)ntx * nty * nzc * nshots;
  const int64_t nblk8 = ((nblk + 7) / 8) * 8;
  int64_t L = xcd_remap(blockIdx.x, nblk8);
  if (L >= nblk) return;
  const int bxi = (int)(L % ntx);
  L /= ntx;
  const int byi = (int)(L % nty);
  L /= nty;
  const int bzi = (int)(L % nzc);
  const int shot = (int)(L / nzc);
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int x0 = bxi * TX, y0 = byi * TY;
  const int z0 = bzi * zchunk, z1 = min(nz, z0 + zchunk);
  const int64_t plane = pitch * ny;
  const T *u = un + (size_t)shot * vol;
  T *o = um + (size_t)shot * vol;
  T *od = DL ? dd + (size_t)shot * vol : nullptr;
  const int xg = x0 + tx;
  const int xw = xg % nx;
  const bool xin = xg < nx;
  int yw[RY];
  bool yin[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    int yg = y0 + ty * RY + r;
    yin[r] = yg < ny;
    yw[r] = yg % ny;
  }
  T q[RY][2 * H + 1];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
#pragma unroll
    for (int k = 0; k < 2 * H; ++k) {
      int z = z0 - H + k;
      q[r][k] = (z >= 0 && z < nz) ? u[(size_t)z * plane + (size_t)yw[r] * pitch + xw] : T(0);
    }
  }
  // halo coordinates owned by this thread
  const int t = threadIdx.x;
  int hy_row[2], hy_x[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    int idx = t + i * 256;            // 2H rows x 64 columns (H <= 4)
    int hr = idx / TX, hc = idx % TX;
    int yg = (hr < H) ? y0 - H + hr : y0 + TY + (hr - H);
    hy_row[i] = (hr < 2 * H) ? ((yg % ny) + ny) % ny : -1;
    hy_x[i] = hc;
  }
  const bool xl = tx < H, xr = tx >= TX - H;
  const int xh = xl ? ((x0 - H + tx) % nx + nx) % nx : (xr ? (x0 + TX + (tx - (TX - H))) % nx : 0);
  const int lxh = xl ? tx : (xr ? TX + H + (tx - (TX - H)) : 0);
  for (int z = z0; z < z1; ++z) {
    const size_t zoff = (size_t)z * plane;
    // next plane of the queue and the centre values of p^{n-1} and K (in flight early)
    T nxt[RY], pm[RY], kk[RY];
    const int zn = z + H;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      nxt[r] = (zn < nz) ? u[(size_t)zn * plane + (size_t)yw[r] * pitch + xw] : T(0);
      size_t c = zoff + (size_t)yw[r] * pitch + xw;
      pm[r] = DL ? od[c] : o[c];
      kk[r] = K[c];
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) q[r][2 * H] = nxt[r];
#pragma unroll
    for (int r = 0; r < RY; ++r) tile[H + ty * RY + r][H + tx] = q[r][H];
    if (xl || xr) {
#pragma unroll
      for (int r = 0; r < RY; ++r) tile[H + ty * RY + r][lxh] = u[zoff + (size_t)yw[r] * pitch + xh];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      if (hy_row[i] >= 0) {
        int hr = (t + i * 256) / TX;
        int ly = (hr < H) ? hr : TY + H + (hr - H);
        int xx = (x0 + hy_x[i]) % nx;
        tile[ly][H + hy_x[i]] = u[zoff + (size_t)hy_row[i] * pitch + xx];
      }
    }
    __syncthreads();
    const T sxz = sx[xw] + sz[z];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int ly = H + ty * RY + r, lx = H + tx;
      const T c = q[r][H];
      const T s = sxz + sy[yw[r]];
      if constexpr (DL) {
        const T lap = lap_diff<H>(W, c, [&](int k, int side) {
          return side == 0 ? tile[ly][lx - k] : side == 1 ? tile[ly][lx + k]
               : side == 2 ? tile[ly - k][lx] : side == 3 ? tile[ly + k][lx]
               : side == 4 ? q[r][H - k] : q[r][H + k];
        });
        const T d = increment(kk[r], lap, pm[r], s);
        if (xin && yin[r]) {
          const size_t g = zoff + (size_t)yw[r] * pitch + xw;
          od[g] = d;
          o[g] = c + d;
        }
      } else {
        T lap = T(3) * W.w[0] * c;
#pragma unroll
        for (int k = 1; k <= H; ++k)
          lap += W.w[k] * ((tile[ly][lx - k] + tile[ly][lx + k]) + (tile[ly - k][lx] + tile[ly + k][lx]) +
                           (q[r][H - k] + q[r][H + k]));
        if (xin && yin[r]) o[zoff + (size_t)yw[r] * pitch + xw] = (T(2) * c - (T(1) - s) * pm[r] + kk[r] * lap) / (T(1) + s);
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RY; ++r) {
#pragma unroll
      for (int k = 0; k < 2 * H; ++k) q[r][k] = q[r][k + 1];
    }
  }
}

// ---- 3D interior, software-pipelined ---------------------------------------------
// Same tiling as k_interior3d, but everything plane z+1 needs from memory (the queue's
// new plane, p^{n-1}, K and the LDS halo of the centre plane) is requested during plane
// z, and the LDS centre plane is double buffered so one barrier per plane suffices.
template <typename T, int H, int RY, int NW, bool DL>
__launch_bounds__(64 * NW)
__global__ void k_interior3d_p(const T *__restrict__ un, T *__restrict__ um, T *__restrict__ dd, const T *__restrict__ K,
                               const T *__restrict__ sx, const T *__restrict__ sy, const T *__restrict__ sz,
                               StencilW<T> W, StencilW<double> WD, int nx, int ny, int nz, int64_t pitch, int64_t vol,
                               int zchunk, int ntx, int nty, int nzc, int nshots, const int2 *__restrict__ zrange) {
  constexpr int TX = 64, TY = NW * RY, LX = TX + 2 * H, LY = TY + 2 * H;
  __shared__ T tile[2][LY][LX];
  const int64_t nblk = (int64_t)ntx * nty * nzc * nshots;
  // tiles in plain launch order, dealt round-robin to the XCDs: the XCD-aware order
  // (xcd_remap), which keeps neighbouring tiles and their halos in one L2, raised the L2 hit
  // rate from 24 % to 39 % but ran 5 % slower on the 401 x 401 x 301 workload
  int64_t L = blockIdx.x;
  if (L >= nblk) return;
  const int bxi = (int)(L % ntx);
  L /= ntx;
  const int byi = (int)(L % nty);
  L /= nty;
  const int bzi = (int)(L % nzc);
  const int shot = (int)(L / nzc);
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int x0 = bxi * TX, y0 = byi * TY;
  // planes of the tile's columns outside [zrange.x, zrange.y) hold exterior nodes only,
  // whose values stay zero: the tile's nzc chunks split that range evenly, so that the
  // blocks of shallow and deep tiles carry the same work
  (void)zchunk;                               // the host derives nzc from it
  const int2 zr = zrange[byi * ntx + bxi];
  const int zcs = (zr.y - zr.x + nzc - 1) / nzc;
  const int z0 = zr.x + bzi * zcs, z1 = min(zr.y, z0 + zcs);
  if (z0 >= z1) return;
  // 32-bit element offsets inside one shot's volume (the launcher checks the volume fits),
  // so that addresses are a scalar base plus one 32-bit offset
  const uint32_t plane = (uint32_t)(pitch * ny);
  const T *u = un + (size_t)shot * vol;
  T *o = um + (size_t)shot * vol;
  // p^{n-1} (plain) or d^n (increment form) at the centre: read once per node
  const T *pin = DL ? dd + (size_t)shot * vol : o;
  T *od = DL ? dd + (size_t)shot * vol : nullptr;
  const int xg = x0 + tx;
  const int xw = xg % nx;
  const bool xin = xg < nx;
  // the edge tiles' lanes past the grid: those within H of it hold the wrapped centre
  // values that the last columns and rows read as neighbours; the others load nothing
  const bool xld = xg < nx + H;
  uint32_t rowoff[RY];
  bool yin[RY], cin[RY], pld[RY];
  int ywv[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    int yg = y0 + ty * RY + r;
    yin[r] = yg < ny;
    cin[r] = xin && yin[r];
    pld[r] = xld && yg < ny + H;
    ywv[r] = yg % ny;
    rowoff[r] = (uint32_t)ywv[r] * (uint32_t)pitch + (uint32_t)xw;
  }
  // halo sources of this thread (x halo: up to RY values; y halo: 2 values)
  const bool xl = tx < H, xr = tx >= TX - H;
  const int xh = xl ? ((x0 - H + tx) % nx + nx) % nx : (xr ? (x0 + TX + (tx - (TX - H))) % nx : 0);
  const int lxh = xl ? tx : (xr ? TX + H + (tx - (TX - H)) : 0);
  constexpr int NHY = (2 * H * TX + 64 * NW - 1) / (64 * NW);   // y-halo values per thread
  uint32_t hyoff[NHY];
  int hyly[NHY], hylx[NHY];
  bool hyon[NHY];
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < NHY; ++i) {
    int idx = t + i * 64 * NW;
    // every thread holds NHY halo values when the halo divides evenly (no predicate)
    hyon[i] = ((2 * H * TX) % (64 * NW) == 0) || idx < 2 * H * TX;
    if (!hyon[i]) idx = 0;
    int hr = idx / TX, hc = idx % TX;
    int yg = (hr < H) ? y0 - H + hr : y0 + TY + (hr - H);
    int yy = ((yg % ny) + ny) % ny;
    hyoff[i] = (uint32_t)yy * (uint32_t)pitch + (uint32_t)((x0 + hc) % nx);
    hyly[i] = (hr < H) ? hr : TY + H + (hr - H);
    hylx[i] = H + hc;
  }
  T q[RY][2 * H + 1];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
#pragma unroll
    for (int k = 0; k <= 2 * H; ++k) {
      int z = z0 - H + k;
      q[r][k] = (z >= 0 && z < nz && pld[r]) ? u[(uint32_t)z * plane + rowoff[r]] : T(0);
    }
  }
  T pm[RY], kk[RY], hx[RY], hy[NHY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    pm[r] = cin[r] ? pin[(uint32_t)z0 * plane + rowoff[r]] : T(0);
    kk[r] = cin[r] ? K[(uint32_t)z0 * plane + rowoff[r]] : T(0);
    hx[r] = (xl || xr) ? u[(uint32_t)z0 * plane + (uint32_t)ywv[r] * (uint32_t)pitch + (uint32_t)xh] : T(0);
  }
#pragma unroll
  for (int i = 0; i < NHY; ++i) hy[i] = hyon[i] ? u[(uint32_t)z0 * plane + hyoff[i]] : T(0);
  int buf = 0;
  for (int z = z0; z < z1; ++z) {
    // centre plane and its halo into LDS
#pragma unroll
    for (int r = 0; r < RY; ++r) tile[buf][H + ty * RY + r][H + tx] = q[r][H];
    if (xl || xr) {
#pragma unroll
      for (int r = 0; r < RY; ++r) tile[buf][H + ty * RY + r][lxh] = hx[r];
    }
#pragma unroll
    for (int i = 0; i < NHY; ++i)
      if (hyon[i]) tile[buf][hyly[i]][hylx[i]] = hy[i];
    // requests for the next plane
    T nq[RY], npm[RY], nk[RY], nhx[RY], nhy[NHY];
    const int zn = z + 1;
    const bool more = zn < z1;
    const uint32_t znoff = (uint32_t)zn * plane;
    const int zq = z + H + 1;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      nq[r] = (zq < nz && pld[r]) ? u[(uint32_t)zq * plane + rowoff[r]] : T(0);
      // p^{n-1} and K are read once: non-temporal, so that p^n halos keep the caches
      npm[r] = (more && cin[r]) ? __builtin_nontemporal_load(&pin[znoff + rowoff[r]]) : T(0);
      nk[r] = (more && cin[r]) ? __builtin_nontemporal_load(&K[znoff + rowoff[r]]) : T(0);
      nhx[r] = (more && (xl || xr)) ? u[znoff + (uint32_t)ywv[r] * (uint32_t)pitch + (uint32_t)xh] : T(0);
    }
#pragma unroll
    for (int i = 0; i < NHY; ++i) nhy[i] = (more && hyon[i]) ? u[znoff + hyoff[i]] : T(0);
    __syncthreads();
    const T sxz = sx[xw] + sz[z];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int ly = H + ty * RY + r, lx = H + tx;
      const T c = q[r][H];
      const T s = sxz + sy[ywv[r]];
      if constexpr (DL) {
        const T lap = lap_diff<H>(W, c, [&](int k, int side) {
          return side == 0 ? tile[buf][ly][lx - k] : side == 1 ? tile[buf][ly][lx + k]
               : side == 2 ? tile[buf][ly - k][lx] : side == 3 ? tile[buf][ly + k][lx]
               : side == 4 ? q[r][H - k] : q[r][H + k];
        });
        const T d = increment(kk[r], lap, pm[r], s);
        if (xin && yin[r]) {
          const uint32_t g = (uint32_t)z * plane + rowoff[r];
          __builtin_nontemporal_store(d, &od[g]);
          __builtin_nontemporal_store(c + d, &o[g]);
        }
      } else {
        T lap = T(3) * W.w[0] * c;
#pragma unroll
        for (int k = 1; k <= H; ++k)
          lap += W.w[k] * ((tile[buf][ly][lx - k] + tile[buf][ly][lx + k]) +
                           (tile[buf][ly - k][lx] + tile[buf][ly + k][lx]) + (q[r][H - k] + q[r][H + k]));
        if (xin && yin[r])
          __builtin_nontemporal_store((T(2) * c - (T(1) - s) * pm[r] + kk[r] * lap) / (T(1) + s),
                                      &o[(uint32_t)z * plane + rowoff[r]]);
      }
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) {
#pragma unroll
      for (int k = 0; k < 2 * H; ++k) q[r][k] = q[r][k + 1];
      q[r][2 * H] = nq[r];
      pm[r] = npm[r];
      kk[r] = nk[r];
      hx[r] = nhx[r];
    }
#pragma unroll
    for (int i = 0; i < NHY; ++i) hy[i] = nhy[i];
    buf ^= 1;
  }
}

// ---- generic interior (2D, or 3D with other orders): one thread per node ------------
template <typename T, int H, bool DL>
__global__ void k_interior_generic(const T *__restrict__ un, T *__restrict__ um, T *__restrict__ dd,
                                   const T *__restrict__ K,
                                   const T *__restrict__ sx, const T *__restrict__ sy, const T *__restrict__ sz,
                                   StencilW<T> W, StencilW<double> WD, int nx, int ny, int nz, int lat,
                                   int64_t pitch, int64_t vol, int nshots, int zf, int zl) {
  // only the planes [zf, zl) hold interior nodes; the others hold zeros that stay zero
  const int64_t per = (int64_t)nx * ny * (zl - zf);
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= per * nshots) return;
  const int shot = (int)(g / per);
  int64_t i = g % per;
  const int x = (int)(i % nx);
  i /= nx;
  const int y = (int)(i % ny);
  const int z = zf + (int)(i / ny);
  const int64_t plane = pitch * ny;
  const T *u = un + (size_t)shot * vol;
  T *o = um + (size_t)shot * vol;
  const size_t c = (size_t)z * plane + (size_t)y * pitch + x;
  const T uc = u[c];
  const T s = sx[x] + sy[y] + sz[z];
  if constexpr (DL) {
    // the increment form's difference Laplacian (see lap_diff); nodes beyond the top and
    // the bottom of the box hold zero
    T lap = T(0);
    for (int k = 1; k <= H; ++k) {
      T acc = (u[(size_t)z * plane + (size_t)y * pitch + wrapk(x - k, nx)] - uc) +
              (u[(size_t)z * plane + (size_t)y * pitch + wrapk(x + k, nx)] - uc);
      if (lat == 2)
        acc += (u[(size_t)z * plane + (size_t)wrapk(y - k, ny) * pitch + x] - uc) +
               (u[(size_t)z * plane + (size_t)wrapk(y + k, ny) * pitch + x] - uc);
      acc += ((z - k >= 0 ? u[c - (size_t)k * plane] : T(0)) - uc) + ((z + k < nz ? u[c + (size_t)k * plane] : T(0)) - uc);
      lap = fma(W.w[k], acc, lap);
    }
    T *od = dd + (size_t)shot * vol;
    const T d = increment(K[c], lap, od[c], s);
    od[c] = d;
    o[c] = uc + d;
    return;
  }
  T lap = T(lat + 1) * W.w[0] * uc;
  for (int k = 1; k <= H; ++k) {
    T acc = u[(size_t)z * plane + (size_t)y * pitch + wrapk(x - k, nx)] +
            u[(size_t)z * plane + (size_t)y * pitch + wrapk(x + k, nx)];
    if (lat == 2)
      acc += u[(size_t)z * plane + (size_t)wrapk(y - k, ny) * pitch + x] +
             u[(size_t)z * plane + (size_t)wrapk(y + k, ny) * pitch + x];
    if (z - k >= 0) acc += u[c - (size_t)k * plane];
    if (z + k < nz) acc += u[c + (size_t)k * plane];
    lap += W.w[k] * acc;
  }
  o[c] = (T(2) * uc - (T(1) - s) * o[c] + K[c] * lap) / (T(1) + s);
}

// ---- IB patch: one wavefront per IB point ------------------------------------------
// Per point: one packed record (position, radius code, record offset, scale).  The
// wavefront loads the data-membership mask words of the support ball once, then, in
// groups of 8 x 64 lattice points, computes every lane's weight index (ballot + prefix
// popcount) and gather address first and only then issues all gathers and weight loads,
// so a point costs two dependent memory latencies instead of one per 64 lattice points.
// Away from the lateral edges a precomputed linear offset table (per radius, for this
// layout) replaces the periodic wrap.
template <typename T>
struct alignas(16) PInfo {
  int16_t x, y, z, code;
  uint32_t roff;
  uint32_t pad;
  T scale;
};

template <typename T, int G>
__device__ __forceinline__ void patch_group(const T *__restrict__ u, const T *__restrict__ wts,
                                            const int32_t *__restrict__ bl, const int32_t *__restrict__ dl,
                                            uint32_t mw, int g0, int nb, int lane, bool edge, int x, int y, int z,
                                            int nx, int ny, int64_t pitch, int64_t plane, size_t centre, int &wbase,
                                            T &acc) {
  int widx[G];
  int64_t gofs[G];
  bool ok[G];
#pragma unroll
  for (int k = 0; k < G; ++k) {
    const int b = (g0 + k) * 64 + lane;
    const uint32_t word = (uint32_t)__shfl((int)mw, (b >> 5) & 63);
    const int bit = (b < nb) ? (int)((word >> (b & 31)) & 1u) : 0;
    const unsigned long long bal = __ballot(bit);
    widx[k] = wbase + __popcll(bal & ((1ull << lane) - 1ull));
    wbase += __popcll(bal);
    ok[k] = bit != 0;
    if (!edge) {
      gofs[k] = (int64_t)centre + (bit ? dl[b] : 0);
    } else {
      const uint32_t v = bit ? (uint32_t)bl[b] : 0u;
      const int dx = (int8_t)(v & 255), dy = (int8_t)((v >> 8) & 255), dz = (int8_t)((v >> 16) & 255);
      gofs[k] = (int64_t)(z + dz) * plane + (int64_t)wrapk(y + dy, ny) * pitch + wrapk(x + dx, nx);
    }
  }
  T pv[G], wv[G];
#pragma unroll
  for (int k = 0; k < G; ++k) {
    pv[k] = ok[k] ? u[gofs[k]] : T(0);
    wv[k] = ok[k] ? wts[widx[k]] : T(0);
  }
#pragma unroll
  for (int k = 0; k < G; ++k) acc += wv[k] * pv[k];
}

// point i of pinfo on one wavefront (every lane of it active)
template <typename T>
__device__ __forceinline__ void gather_point(int64_t i, const T *__restrict__ un, T *__restrict__ unew,
                                             T *__restrict__ dd, const uint32_t *__restrict__ rec,
                                             const PInfo<T> *__restrict__ pinfo, const int32_t *__restrict__ ball,
                                             const int32_t *__restrict__ delta, const int32_t *__restrict__ ball_meta,
                                             int nx, int ny, int64_t pitch, int64_t vol, int nshots) {
  const int lane = threadIdx.x & 63;
  const PInfo<T> P = pinfo[i];
  const int x = P.x, y = P.y, z = P.z, code = P.code;
  const int bstart = ball_meta[2 * code], nb = ball_meta[2 * code + 1];
  const int nwords = (nb + 31) >> 5;
  const uint32_t *m = rec + P.roff;
  const int wpad = (sizeof(T) == 8) ? ((nwords + 1) & ~1) : nwords;
  const T *wts = reinterpret_cast<const T *>(m + wpad);
  const uint32_t mw = (lane < nwords) ? m[lane] : 0u;      // nb <= 2048 -> nwords <= 64
  const int64_t plane = pitch * ny;
  const int R = code / 2 + 1;
  const bool edge = (x < R || x >= nx - R || (ny > 1 && (y < R || y >= ny - R)));
  const size_t centre = (size_t)z * plane + (size_t)y * pitch + x;
  const int32_t *bl = ball + bstart;
  const int32_t *dl = delta + bstart;
  const int ngroups = (nb + 511) / 512;
  for (int s = 0; s < nshots; ++s) {
    const T *u = un + (size_t)s * vol;
    T acc = T(0);
    int wbase = 0;
    for (int g = 0; g < ngroups; ++g)
      patch_group<T, 8>(u, wts, bl, dl, mw, g * 8, nb, lane, edge, x, y, z, nx, ny, pitch, plane, centre, wbase, acc);
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) {
      const T v = mul_rn(P.scale, acc);
      unew[(size_t)s * vol + centre] += v;
      if (dd) dd[(size_t)s * vol + centre] += v;
    }
  }
}

// the gather patch, four points per workgroup, after the workgroups of io (2D)
template <typename T>
__launch_bounds__(256)
__global__ void k_patch(const T *__restrict__ un, T *__restrict__ unew, T *__restrict__ dd,
                        const uint32_t *__restrict__ rec,
                        const PInfo<T> *__restrict__ pinfo, const int32_t *__restrict__ ball,
                        const int32_t *__restrict__ delta, const int32_t *__restrict__ ball_meta, int64_t nib,
                        int nx, int ny, int nz, int64_t pitch, int64_t vol, int nshots, PatchIo<T> io) {
  const int b = (int)blockIdx.x, nsp = io.nsb + io.ninj;
  if (b < io.nsb) {
    sample_block(un, io, b, vol);
    finish_io(io);
    return;
  }
  if (b < nsp) {
    inject_sources(unew, dd, io.sidx, io.sw, nshots, vol, io.wavelet, io.wstride, io.tcount[0]);
    finish_io(io);
    return;
  }
  const int64_t blk = xcd_remap(b - nsp, gridDim.x - nsp);
  const int64_t i = blk * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= nib) return;
  gather_point<T>(i, un, unew, dd, rec, pinfo, ball, delta, ball_meta, nx, ny, pitch, vol, nshots);
}

// ---- IB patch, LDS-tiled (3D) -------------------------------------------------------
// IB points are bucketed into TX x TY x TZ tiles (host, at state creation; laterally
// aligned, in depth starting at the tile's first point).  A workgroup
// stages p^n over its tile plus an HR-cell halo in LDS with coalesced row loads; its
// wavefronts then evaluate the tile's points from LDS, each streaming the point's
// dense-range weights (coalesced, no mask decoding) while the next point's record is
// already in flight.  The support balls of neighbouring points overlap almost entirely,
// so each p^n value is fetched from memory about once per tile.  Points whose support
// radius exceeds HR + 1/2 stay on the gather kernel above.
template <typename T>
struct alignas(16) PInfoD {
  int16_t x, y, z, code;
  uint16_t first, count;
  uint32_t woff;
  T scale;
};

template <typename T, int TX, int TY, int TZ, int HR, int PV>
__launch_bounds__(512)
__global__ void k_patch_tiled(const T *__restrict__ un, T *__restrict__ unew, T *__restrict__ dd,
                              const T *__restrict__ dense,
                              const PInfoD<T> *__restrict__ pinfo, const int32_t *__restrict__ ball,
                              const int32_t *__restrict__ ball_meta, const int4 *__restrict__ tiles, int ntiles,
                              int nx, int ny, int nz, int64_t pitch, int64_t vol, int nshots) {
  // odd row pitch in LDS: the lattice rows of a support ball fall in different banks
  constexpr int LX = TX + 2 * HR + 1, LY = TY + 2 * HR, LZ = TZ + 2 * HR;
  constexpr int NS = 7;                       // 64-lane slots per point (ball of radius 4.5: 389 points)
  constexpr int BMAX = 64 * NS;
  __shared__ T sp[LZ * LY * LX];
  __shared__ int16_t lofs[2][BMAX];           // LDS offsets of the ball lattice points, radius codes 8 and 9
  __shared__ T res[kTileMaxPoints];            // per-point results, written back together
  const int64_t tb = xcd_remap(blockIdx.x, gridDim.x);
  if (tb >= ntiles) return;
  const int4 tl = tiles[tb];
  const int x0 = tl.x, y0 = tl.y, z0 = tl.z;
  const int p0 = tl.w, p1 = tiles[tb + 1].w;
  const int lane = threadIdx.x & 63, nwave = blockDim.x >> 6;
  // the wavefront index is uniform: make it a scalar so that the per-point records are
  // scalar loads and the weight addresses are scalar base + lane offset
  const int wave = (PV & 1) ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : (int)(threadIdx.x >> 6);
  const int64_t plane = pitch * ny;
  for (int q = 0; q < 2; ++q) {
    const int code = 8 + q, st0 = ball_meta[2 * code], nbq = ball_meta[2 * code + 1];
    for (int b = threadIdx.x; b < BMAX; b += blockDim.x) {
      int v = 0;
      if (b < nbq) {
        const uint32_t e = (uint32_t)ball[st0 + b];
        const int dx = (int8_t)(e & 255), dy = (int8_t)((e >> 8) & 255), dz = (int8_t)((e >> 16) & 255);
        v = (dz * LY + dy) * LX + dx;
      }
      lofs[q][b] = (int16_t)v;
    }
  }
  for (int s = 0; s < nshots; ++s) {
    const T *u = un + (size_t)s * vol;
    // software pipeline over this wavefront's points, two at a time: the weights of the
    // next pair and the records of the pair after it are in flight while a pair is
    // evaluated (four points' weights outstanding per wavefront)
    const int step2 = 2 * nwave;
    int p = p0 + wave;
    PInfoD<T> Pc[2], Pn[2];
    T wc[2][NS], wn[2][NS];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = p + h * nwave;
      if (q < p1) Pc[h] = pinfo[q];
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = p + h * nwave;
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const int e = k * 64 + lane;
        wc[h][k] = (q < p1 && e < Pc[h].count) ? dense[Pc[h].woff + e] : T(0);
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = p + step2 + h * nwave;
      if (q < p1) Pn[h] = pinfo[q];
    }
    for (int e = threadIdx.x; e < LZ * LY * LX; e += blockDim.x) {
      const int lx = e % LX, ly = (e / LX) % LY, lz = e / (LX * LY);
      const int gz = z0 - HR + lz;
      const int gx = wrapk(x0 - HR + lx, nx), gy = wrapk(y0 - HR + ly, ny);
      sp[e] = (lx < LX - 1 && gz >= 0 && gz < nz) ? u[(size_t)gz * plane + (size_t)gy * pitch + gx] : T(0);
    }
    __syncthreads();
    while (p < p1) {
      const int pn = p + step2;
      PInfoD<T> Pnn[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int q = pn + h * nwave;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          const int e = k * 64 + lane;
          wn[h][k] = (q < p1 && e < Pn[h].count) ? dense[Pn[h].woff + e] : T(0);
        }
        const int q2 = pn + step2 + h * nwave;
        if (q2 < p1) Pnn[h] = pinfo[q2];
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int q = p + h * nwave;
        if (q < p1) {
          const PInfoD<T> &P = Pc[h];
          int cx = P.x - x0;
          if (cx < 0) cx += nx;
          int cy = P.y - y0;
          if (cy < 0) cy += ny;
          const int lc = ((P.z - z0 + HR) * LY + (cy + HR)) * LX + (cx + HR);
          const int16_t *lt = lofs[P.code == 9 ? 1 : 0] + P.first;
          T acc = T(0);
#pragma unroll
          for (int k = 0; k < NS; ++k) {
            const int e = k * 64 + lane;
            if (e < P.count) acc += wc[h][k] * sp[lc + lt[e]];
          }
          if (PV & 2) {
            acc = wave_sum(acc);
          } else {
            for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
          }
          if (lane == 0) res[q - p0] = P.scale * acc;
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        Pc[h] = Pn[h];
        Pn[h] = Pnn[h];
#pragma unroll
        for (int k = 0; k < NS; ++k) wc[h][k] = wn[h][k];
      }
      p = pn;
    }
    __syncthreads();
    // read-modify-write of p^{n+1} for all points of the tile at once (kept off the
    // per-point path, where its load would wait behind the prefetched weights)
    for (int q = p0 + (int)threadIdx.x; q < p1; q += blockDim.x) {
      const PInfoD<T> P = pinfo[q];
      const size_t g = (size_t)s * vol + (size_t)P.z * plane + (size_t)P.y * pitch + P.x;
      unew[g] += res[q - p0];
      if (dd) dd[g] += res[q - p0];
    }
    __syncthreads();
  }
}

// Same computation with the tile's point records staged in LDS (read back as scalars, so
// no scalar memory load is outstanding while LDS results are awaited), the weights of D
// groups of two points per wavefront in flight, DPP wavefront sums, and the scale applied
// in the per-tile read-modify-write.
struct TileRec {
  uint32_t woff;      // first dense weight
  uint32_t fc;        // first lattice index | count << 16
  uint32_t lcc;       // LDS index of the point | radius code 9 << 31
  uint32_t pad;
};

template <typename T, int NS>
struct PairW {
  T w[2][NS];
};

// VW = 2 (FP32): each lane loads two consecutive weights at once (dense ranges start at
// even offsets and are padded with a zero to an even length), halving the weight loads.
template <typename T, int TX, int TY, int TZ, int HR, int D, int SC, int VW = 1>
__launch_bounds__(512)
__global__ void k_patch_tiled_r(const T *__restrict__ un, T *__restrict__ unew, T *__restrict__ dd,
                                const T *__restrict__ dense,
                                const PInfoD<T> *__restrict__ pinfo, const int32_t *__restrict__ ball,
                                const int32_t *__restrict__ ball_meta, const int4 *__restrict__ tiles, int ntiles,
                                int nx, int ny, int nz, int64_t pitch, int64_t vol, int nshots) {
  constexpr int LX = TX + 2 * HR + 1, LY = TY + 2 * HR, LZ = TZ + 2 * HR;
  constexpr int NS = 7;
  constexpr int BMAX = 64 * NS;
  constexpr int NW = 8;                       // wavefronts per workgroup (512 threads)
  constexpr int STEP = 2 * NW;                // points per wavefront group step
  static_assert(VW == 1 || (VW == 2 && sizeof(T) == 4), "paired weight loads are FP32 only");
  using WT = std::conditional_t<VW == 2, float2, T>;
  constexpr int NSL = (VW == 2) ? 4 : NS;     // load slots per point (64 x VW lattice points each)
  // SC shots per pass: their tiles side by side in LDS, each point's weights loaded once
  __shared__ T sp[SC][LZ * LY * LX];
  __shared__ int16_t lofs[2][BMAX];
  __shared__ TileRec rec[kTileMaxPoints];
  __shared__ T res[SC][kTileMaxPoints];
  const int64_t tb = xcd_remap(blockIdx.x, gridDim.x);
  if (tb >= ntiles) return;
  const int4 tl = tiles[tb];
  const int x0 = tl.x, y0 = tl.y, z0 = tl.z;
  const int p0 = tl.w, np = tiles[tb + 1].w - tl.w;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t plane = pitch * ny;
  for (int q = 0; q < 2; ++q) {
    const int code = 8 + q, st0 = ball_meta[2 * code], nbq = ball_meta[2 * code + 1];
    for (int b = threadIdx.x; b < BMAX; b += blockDim.x) {
      int v = 0;
      if (b < nbq) {
        const uint32_t e = (uint32_t)ball[st0 + b];
        const int dx = (int8_t)(e & 255), dy = (int8_t)((e >> 8) & 255), dz = (int8_t)((e >> 16) & 255);
        v = (dz * LY + dy) * LX + dx;
      }
      lofs[q][b] = (int16_t)v;
    }
  }
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    const PInfoD<T> P = pinfo[p0 + i];
    int cx = P.x - x0;
    if (cx < 0) cx += nx;
    int cy = P.y - y0;
    if (cy < 0) cy += ny;
    const int lc = ((P.z - z0 + HR) * LY + (cy + HR)) * LX + (cx + HR);
    TileRec r;
    r.woff = P.woff;
    r.fc = (uint32_t)P.first | ((uint32_t)P.count << 16);
    r.lcc = (uint32_t)lc | (P.code == 9 ? 0x80000000u : 0u);
    r.pad = 0;
    rec[i] = r;
  }
  __syncthreads();
  auto get = [&](int i, uint32_t &woff, uint32_t &fc, uint32_t &lcc) {
    if (i < np) {
      const TileRec r = rec[i];
      woff = __builtin_amdgcn_readfirstlane(r.woff);
      fc = __builtin_amdgcn_readfirstlane(r.fc);
      lcc = __builtin_amdgcn_readfirstlane(r.lcc);
    } else {
      woff = 0, fc = 0, lcc = 0;           // count 0: nothing loaded, nothing evaluated
    }
  };
  auto load = [&](PairW<WT, NSL> &W, const uint32_t (&wo)[2], const uint32_t (&fc)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int cnt = (int)(fc[h] >> 16);
#pragma unroll
      for (int k = 0; k < NSL; ++k) {
        const int e = (k * 64 + lane) * VW;
        // the weights are streamed once: non-temporal loads measured faster in FP64 and
        // slightly slower in FP32
        if constexpr (VW == 2)
          W.w[h][k] = (e < cnt) ? *reinterpret_cast<const float2 *>(&dense[wo[h] + e]) : float2(0.0f, 0.0f);
        else if constexpr (sizeof(T) == 8)
          W.w[h][k] = (e < cnt) ? __builtin_nontemporal_load(&dense[wo[h] + e]) : T(0);
        else
          W.w[h][k] = (e < cnt) ? dense[wo[h] + e] : T(0);
      }
    }
  };
  for (int s0 = 0; s0 < nshots; s0 += SC) {
    // records of D + 1 groups ahead, weights of D groups in flight before the staging
    uint32_t wo[D + 1][2], fc[D + 1][2], lcc[D + 1][2];
    PairW<WT, NSL> W[D + 1];
#pragma unroll
    for (int d = 0; d <= D; ++d)
#pragma unroll
      for (int h = 0; h < 2; ++h) get(wave + d * STEP + h * NW, wo[d][h], fc[d][h], lcc[d][h]);
#pragma unroll
    for (int d = 0; d < D; ++d) load(W[d], wo[d], fc[d]);
    stage_tile<T, SC, LX, LY, LZ, 512, 1>(&sp[0][0], LZ * LY * LX, un, vol, s0, nshots, x0 - HR, y0 - HR, z0 - HR, nx,
                                       ny, nz, pitch, [](int, int, int) { return true; });
    __syncthreads();
    for (int p = wave; p < np; p += STEP) {
      // weights of the group D steps ahead; its successor's records
      load(W[D], wo[D], fc[D]);
      uint32_t nwo[2], nfc[2], nlcc[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) get(p + (D + 1) * STEP + h * NW, nwo[h], nfc[h], nlcc[h]);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int q = p + h * NW;
        const int cnt = (int)(fc[0][h] >> 16);
        if (cnt > 0) {
          const int first = (int)(fc[0][h] & 0xffffu);
          const int lc = (int)(lcc[0][h] & 0x7fffffffu);
          const int16_t *lt = lofs[lcc[0][h] >> 31] + first;
          T acc[SC];
#pragma unroll
          for (int c = 0; c < SC; ++c) acc[c] = T(0);
#pragma unroll
          for (int k = 0; k < NSL; ++k) {
            const int e = (k * 64 + lane) * VW;
            if (e < cnt) {
              if constexpr (VW == 2) {
                // e + 1 <= count: a zero weight at the record's pad, its lattice index in range
                const int o0 = lc + lt[e], o1 = lc + lt[e + 1];
                // explicit fused multiply-adds: every shot count rounds alike
#pragma unroll
                for (int c = 0; c < SC; ++c) acc[c] = fmaf(W[0].w[h][k].y, sp[c][o1], fmaf(W[0].w[h][k].x, sp[c][o0], acc[c]));
              } else {
                const int o = lc + lt[e];
#pragma unroll
                for (int c = 0; c < SC; ++c) acc[c] = fma(W[0].w[h][k], sp[c][o], acc[c]);
              }
            }
          }
#pragma unroll
          for (int c = 0; c < SC; ++c) {
            const T t = wave_sum(acc[c]);
            if (lane == 0) res[c][q] = t;
          }
        }
      }
#pragma unroll
      for (int d = 0; d < D; ++d) {
        W[d] = W[d + 1];
#pragma unroll
        for (int h = 0; h < 2; ++h) wo[d][h] = wo[d + 1][h], fc[d][h] = fc[d + 1][h], lcc[d][h] = lcc[d + 1][h];
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) wo[D][h] = nwo[h], fc[D][h] = nfc[h], lcc[D][h] = nlcc[h];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
      const PInfoD<T> P = pinfo[p0 + i];
      const size_t g = (size_t)P.z * plane + (size_t)P.y * pitch + P.x;
#pragma unroll
      for (int c = 0; c < SC; ++c)
        if (s0 + c < nshots) {
          const T v = mul_rn(P.scale, res[c][i]);
          unew[(size_t)(s0 + c) * vol + g] += v;
          if (dd) dd[(size_t)(s0 + c) * vol + g] += v;
        }
    }
    __syncthreads();
  }
}

// Tiled patch streaming the compact records (bit mask of the support ball's data nodes,
// then the weights of the set bits): only the weights of data nodes cross HBM.  A point's
// mask words arrive one group ahead of its weights; each 64-lattice-point slot's word is
// read into scalars, a lane's weight index is the count of set bits below it plus the
// slot's base, and the lanes' LDS offsets for the two tiled ball sizes sit in registers.
struct TileRecM {
  uint32_t roff;      // record offset (32-bit words)
  uint32_t lcc;       // LDS index of the point | radius code 9 << 31
};

template <typename T, int TX, int TY, int TZ, int HR>
__launch_bounds__(512)
__global__ void k_patch_tiled_m(const T *__restrict__ un, T *__restrict__ unew, T *__restrict__ dd,
                                const uint32_t *__restrict__ rec,
                                const PInfo<T> *__restrict__ pinfo, const int32_t *__restrict__ ball,
                                const int32_t *__restrict__ ball_meta, const int4 *__restrict__ tiles, int ntiles,
                                int nx, int ny, int nz, int64_t pitch, int64_t vol, int nshots) {
  constexpr int LX = TX + 2 * HR + 1, LY = TY + 2 * HR, LZ = TZ + 2 * HR;
  constexpr int NS = 7;                       // 64-lattice-point slots (balls of up to 448 points)
  constexpr int NW = 8;
  constexpr int STEP = 2 * NW;
  __shared__ T sp[LZ * LY * LX];
  __shared__ TileRecM trec[kTileMaxPoints];
  __shared__ T res[kTileMaxPoints];
  const int64_t tb = xcd_remap(blockIdx.x, gridDim.x);
  if (tb >= ntiles) return;
  const int4 tl = tiles[tb];
  const int x0 = tl.x, y0 = tl.y, z0 = tl.z;
  const int p0 = tl.w, np = tiles[tb + 1].w - tl.w;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t plane = pitch * ny;
  // ball codes 8 and 9: sizes, mask words, weight start (FP64 weights are 8-byte aligned)
  int nbc[2], nwc[2], wpc[2];
  int lo[2][NS];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int code = 8 + q, st0 = ball_meta[2 * code];
    nbc[q] = ball_meta[2 * code + 1];
    nwc[q] = (nbc[q] + 31) >> 5;
    wpc[q] = (sizeof(T) == 8) ? ((nwc[q] + 1) & ~1) : nwc[q];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const int b = k * 64 + lane;
      int v = 0;
      if (b < nbc[q]) {
        const uint32_t e = (uint32_t)ball[st0 + b];
        const int dx = (int8_t)(e & 255), dy = (int8_t)((e >> 8) & 255), dz = (int8_t)((e >> 16) & 255);
        v = (dz * LY + dy) * LX + dx;
      }
      lo[q][k] = v;
    }
  }
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    const PInfo<T> P = pinfo[p0 + i];
    int cx = P.x - x0;
    if (cx < 0) cx += nx;
    int cy = P.y - y0;
    if (cy < 0) cy += ny;
    const int lc = ((P.z - z0 + HR) * LY + (cy + HR)) * LX + (cx + HR);
    TileRecM r;
    r.roff = P.roff;
    r.lcc = (uint32_t)lc | (P.code == 9 ? 0x80000000u : 0u);
    trec[i] = r;
  }
  __syncthreads();
  auto get = [&](int i, uint32_t &roff, uint32_t &lcc) {
    if (i < np) {
      const TileRecM r = trec[i];
      roff = __builtin_amdgcn_readfirstlane(r.roff);
      lcc = __builtin_amdgcn_readfirstlane(r.lcc);
    } else {
      roff = 0u, lcc = 0xffffffffu;          // no point
    }
  };
  // the mask words of a point, one per lane (lanes beyond the word count read nothing)
  auto load_mask = [&](uint32_t roff, uint32_t lcc) -> uint32_t {
    if (lcc == 0xffffffffu) return 0u;
    const int nwd = nwc[lcc >> 31];
    return lane < nwd ? rec[roff + lane] : 0u;
  };
  // the weights of a point from its mask (all lanes take part in the scalar reads)
  auto load_w = [&](T (&w)[NS], uint32_t mk, uint32_t roff, uint32_t lcc) {
    const bool live = lcc != 0xffffffffu;
    const int q = (int)(lcc >> 31) & 1;
    const T *wts = reinterpret_cast<const T *>(rec + roff + (live ? wpc[q] : 0));
    uint32_t base = 0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const uint32_t wl = (uint32_t)__builtin_amdgcn_readlane((int)mk, 2 * k);
      const uint32_t wh = (uint32_t)__builtin_amdgcn_readlane((int)mk, 2 * k + 1);
      const uint32_t word = lane < 32 ? wl : wh;
      const bool on = live && ((word >> (lane & 31)) & 1u);
      const uint32_t rank = __builtin_amdgcn_mbcnt_hi(wh, __builtin_amdgcn_mbcnt_lo(wl, 0u));
      w[k] = on ? wts[base + rank] : T(0);
      base += (uint32_t)(__builtin_popcount(wl) + __builtin_popcount(wh));
    }
  };
  for (int s = 0; s < nshots; ++s) {
    const T *u = un + (size_t)s * vol;
    // group g = points (p, p + NW); records two groups ahead, masks one group ahead
    uint32_t ro0[2], lc0[2], ro1[2], lc1[2], ro2[2], lc2[2], mk1[2];
    T w0[2][NS];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      get(wave + h * NW, ro0[h], lc0[h]);
      get(wave + STEP + h * NW, ro1[h], lc1[h]);
      get(wave + 2 * STEP + h * NW, ro2[h], lc2[h]);
    }
    {
      uint32_t mk0[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) mk0[h] = load_mask(ro0[h], lc0[h]);
#pragma unroll
      for (int h = 0; h < 2; ++h) mk1[h] = load_mask(ro1[h], lc1[h]);
#pragma unroll
      for (int h = 0; h < 2; ++h) load_w(w0[h], mk0[h], ro0[h], lc0[h]);
    }
    for (int e = threadIdx.x; e < LZ * LY * LX; e += blockDim.x) {
      const int lx = e % LX, ly = (e / LX) % LY, lz = e / (LX * LY);
      const int gz = z0 - HR + lz;
      const int gx = wrapk(x0 - HR + lx, nx), gy = wrapk(y0 - HR + ly, ny);
      sp[e] = (lx < LX - 1 && gz >= 0 && gz < nz) ? u[(size_t)gz * plane + (size_t)gy * pitch + gx] : T(0);
    }
    __syncthreads();
    for (int p = wave; p < np; p += STEP) {
      // masks of the group two ahead, weights of the next group
      uint32_t mk2[2];
      T w1[2][NS];
#pragma unroll
      for (int h = 0; h < 2; ++h) mk2[h] = load_mask(ro2[h], lc2[h]);
#pragma unroll
      for (int h = 0; h < 2; ++h) load_w(w1[h], mk1[h], ro1[h], lc1[h]);
      uint32_t ro3[2], lc3[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) get(p + 3 * STEP + h * NW, ro3[h], lc3[h]);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (lc0[h] != 0xffffffffu) {
          const int lcx = (int)(lc0[h] & 0x7fffffffu);
          const bool c9 = (lc0[h] >> 31) != 0u;
          T acc = T(0);
#pragma unroll
          for (int k = 0; k < NS; ++k) acc += w0[h][k] * sp[lcx + (c9 ? lo[1][k] : lo[0][k])];
          acc = wave_sum(acc);
          if (lane == 0) res[p + h * NW] = acc;
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        ro0[h] = ro1[h], lc0[h] = lc1[h];
        ro1[h] = ro2[h], lc1[h] = lc2[h];
        ro2[h] = ro3[h], lc2[h] = lc3[h];
        mk1[h] = mk2[h];
#pragma unroll
        for (int k = 0; k < NS; ++k) w0[h][k] = w1[h][k];
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
      const PInfo<T> P = pinfo[p0 + i];
      const size_t g = (size_t)s * vol + (size_t)P.z * plane + (size_t)P.y * pitch + P.x;
      const T v = mul_rn(P.scale, res[i]);
      unew[g] += v;
      if (dd) dd[g] += v;
    }
    __syncthreads();
  }
}

// Tiled patch streaming the column-run records: only the data nodes' weights cross HBM
// (plus a zero at the rare non-data node inside a column's run).  Lane c of the wavefront
// that evaluates a point takes ball column c (lanes 0..4 also one single-node extra column
// of the radius-4.5 ball): it finds the column's run from the tile's table of first data
// planes, its entries' offset by a prefix sum over the lanes (DPP), and loads a window of
// entries that ends with its run, so that window row k always pairs with the same plane
// (the bottom of the column minus 8 - k): the reads of p^n are one LDS address plus
// immediate offsets, and window rows before the run are dropped with one select each.
// p^n is staged plane by plane with a plane of 256 nodes (bank = column, whatever the
// plane) under four zero planes.  The kernel keeps the vector instructions per point few:
// the table streams at HBM rate only if the wavefronts keep up.  Two points per
// wavefront are in flight (the loads of one while the other is evaluated).  Staging skips
// the nodes above each column's first data plane (their weights are all zero).
struct ColDec {
  int base, mlen, ebase, elen;  // LDS index of the window's first row, run length; extra node, 0/1
  uint32_t off;                 // entry of window row 0 (the run's first entry at row 9 - mlen)
};

// the points of tile tb (one 512-thread workgroup)
template <typename T, int SC>
__device__ __forceinline__ void patch_tile(int64_t tb, const T *__restrict__ un, T *__restrict__ unew,
                                           T *__restrict__ dd, const T *__restrict__ wcol,
                                           const uint2 *__restrict__ recs, const T *__restrict__ scale,
                                           const int16_t *__restrict__ zfirst, const int32_t *__restrict__ coltab,
                                           const int4 *__restrict__ tiles, int nx, int ny, int nz, int64_t pitch,
                                           int64_t vol, int nshots) {
  constexpr int TX = kTileX, TY = kTileY, TZ = kTileZ, HR = kTileHalo;
  constexpr int CX = TX + 2 * HR, CY = TY + 2 * HR, LZ = TZ + 2 * HR;
  constexpr int NE = 2 * HR + 1;          // window rows (the longest column)
  constexpr int NC = CX * CY;             // columns of the tile with its halo
  // LDS layout of the staged planes: rows RP apart, planes PL apart.  The lanes of a point
  // read one plane of their columns at a time, at (half height) * PL + dy * RP + dx from a
  // common base.  Two FP32 shots or FP64 values per node (8 bytes, half as many distinct
  // banks) use 18 x 288, which spreads a ball's columns over the banks with fewer conflicts
  // than the dense 16 x 256 plane and still leaves room for two workgroups per CU; the
  // single FP32 shot keeps the dense plane (its time does not depend on the layout)
  constexpr bool kWide = SC == 2 || sizeof(T) == 8;
  constexpr int RP = kWide ? 18 : CX, PL = kWide ? 288 : NC;
  static_assert(RP >= CX && PL >= RP * CY, "padded layout holds the tile");
  constexpr int ZT = NE - 1 - HR;         // zero planes above the tile (window rows of short columns)
  constexpr int NW = 8;                   // wavefronts per workgroup
  constexpr int VEC = 16 / sizeof(T);     // entries per 16-byte load
  constexpr int NWIN = NE + 1;            // window entries used: rows, then the extra node
  constexpr int NL = (NWIN + VEC - 1) / VEC;
  static_assert(HR == 4 && NC % 64 == 0, "column tables of radius 4 and 4.5; planes of whole bank rows");
  // two FP32 shots sit side by side per node (one 8-byte LDS read for both)
  constexpr bool ILV = SC == 2 && sizeof(T) == 4;
  __shared__ __align__(16) T sp[SC * (ZT + LZ) * PL];
  auto at = [&](int c, int node) -> int { return ILV ? node * SC + c : c * (ZT + LZ) * PL + node; };
  __shared__ int zf[NC];                  // first data plane of each column (tile plane index)
  __shared__ uint2 rec[kTileMaxPoints];   // entry offset; x | y << 5 | z << 10 | radius code 9 << 31
  __shared__ T res[SC][kTileMaxPoints];
  const int4 tl = tiles[tb];
  const int x0 = tl.x, y0 = tl.y, z0 = tl.z;
  const int p0 = tl.w, np = tiles[tb + 1].w - tl.w;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t plane = pitch * ny;
  // this lane's columns as offsets in zf (co = dy * CX + dx) and in an LDS plane (cs = dy *
  // RP + dx), with their half height zr (-1: no column): radius 4.5, radius 4, and the extra
  // column
  int co9, cs9, zr9, co8, cs8, zr8, coe, cse;
  bool hase;
  {
    auto unpack = [&](int32_t col, int &co, int &cs, int &zr) {
      const int dx = (int8_t)(col & 255), dy = (int8_t)((col >> 8) & 255);
      co = col == kNoColumn ? 0 : dy * CX + dx;
      cs = col == kNoColumn ? 0 : dy * RP + dx;
      zr = col == kNoColumn ? -1 : (col >> 16) & 255;
    };
    unpack(coltab[lane], co9, cs9, zr9);
    unpack(lane < kColumns8 ? coltab[kColumns9 + lane] : kNoColumn, co8, cs8, zr8);
    const int32_t e9 = lane < kColumns9 - 64 ? coltab[64 + lane] : kNoColumn;
    int zre;
    unpack(e9, coe, cse, zre);
    hase = e9 != kNoColumn;
  }
  for (int e = threadIdx.x; e < NC; e += blockDim.x) {
    const int gx = wrapk(x0 - HR + e % CX, nx), gy = wrapk(y0 - HR + e / CX, ny);
    zf[e] = (int)zfirst[(int64_t)gy * nx + gx] - (z0 - HR);
  }
  for (int i = threadIdx.x; i < np; i += blockDim.x) rec[i] = recs[p0 + i];
  for (int e = threadIdx.x; e < ZT * PL; e += blockDim.x)
#pragma unroll
    for (int c = 0; c < SC; ++c) sp[at(c, e)] = T(0);
  __syncthreads();
  auto decode = [&](int i) {
    ColDec D{0, 0, 0, 0, 0u};
    // past the tile's points: a point at the tile centre without entries (every window,
    // read and dropped, inside the table's leading padding)
    uint32_t woff = (uint32_t)kColPad, loc = (uint32_t)(HR | (HR << 5) | (HR << 10));
    if (i < np) {
      const uint2 r = rec[i];
      woff = (uint32_t)__builtin_amdgcn_readfirstlane((int)r.x);
      loc = (uint32_t)__builtin_amdgcn_readfirstlane((int)r.y);
    }
    const int lx = (int)(loc & 31), ly = (int)((loc >> 5) & 31), lz = (loc >> 10) & 63;
    const int col = ly * CX + lx, cols = ly * RP + lx;
    const bool is9 = (loc >> 31) != 0u;
    const int co = is9 ? co9 : co8, cs = is9 ? cs9 : cs8, zr = (i < np) ? (is9 ? zr9 : zr8) : -1;
    D.mlen = max(min(zr - zf[col + co] + lz + 1, 2 * zr + 1), 0);
    // window row k: plane lz + zr - 8 + k (a lane without a column reads the top zero plane)
    D.base = (zr >= 0 ? lz + zr - (NE - 1) + ZT : 0) * PL + cols + cs;
    D.elen = (is9 && hase && zf[col + coe] <= lz) ? 1 : 0;
    D.ebase = (lz + ZT) * PL + cols + cse;
    const int len = D.mlen + D.elen;
    D.off = woff + (uint32_t)(wave_incl_scan(len) - len) + (uint32_t)D.mlen - (uint32_t)NE;
    return D;
  };
  // straight-line loads (no branch around a load, so the loads of the next point stay in
  // flight while this one is evaluated); the window's entries outside this lane's own are
  // read and not used (the table has padding before its first and after its last entry)
  auto load = [&](const ColDec &D, T(&w)[NL * VEC]) {
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      if constexpr (VEC == 4) {
        float4 v;
        __builtin_memcpy(&v, wcol + D.off + j * VEC, sizeof(v));
        w[j * VEC] = v.x, w[j * VEC + 1] = v.y, w[j * VEC + 2] = v.z, w[j * VEC + 3] = v.w;
      } else {
        double2 v;
        __builtin_memcpy(&v, wcol + D.off + j * VEC, sizeof(v));
        w[j * VEC] = v.x, w[j * VEC + 1] = v.y;
      }
    }
  };
  auto eval = [&](const ColDec &D, const T(&w)[NL * VEC], int q) {
    T acc[SC];
#pragma unroll
    for (int c = 0; c < SC; ++c) acc[c] = T(0);
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const T wk = (k >= NE - D.mlen) ? w[k] : T(0);
      if constexpr (ILV) {
        float2 pv;
        __builtin_memcpy(&pv, &sp[(D.base + k * PL) * 2], 8);
        acc[0] = fma(wk, pv.x, acc[0]);
        acc[1] = fma(wk, pv.y, acc[1]);
      } else {
#pragma unroll
        for (int c = 0; c < SC; ++c) acc[c] = fma(wk, sp[at(c, D.base + k * PL)], acc[c]);
      }
    }
    const T we = D.elen ? w[NE] : T(0);
#pragma unroll
    for (int c = 0; c < SC; ++c) acc[c] = fma(we, sp[at(c, D.ebase)], acc[c]);
#pragma unroll
    for (int c = 0; c < SC; ++c) {
      const T t = wave_total(acc[c]);
      if (lane == 0 && q < np) res[c][q] = t;
    }
  };
  for (int s0 = 0; s0 < nshots; s0 += SC) {
    // the first point's weights are in flight while the tile is staged
    ColDec D0 = decode(wave), D1;
    T w0[NL * VEC], w1[NL * VEC];
    load(D0, w0);
    auto keep = [&](int lx, int ly, int lz) { return zf[ly * CX + lx] <= lz; };
    stage_tile<T, SC, CX, CY, LZ, 512, 0, decltype(keep), RP, PL, ILV>(&sp[at(0, ZT * PL)], (ZT + LZ) * PL, un, vol,
                                                                       s0, nshots, x0 - HR, y0 - HR, z0 - HR, nx, ny,
                                                                       nz, pitch, keep);
    __syncthreads();
    // points wave, wave + NW, ...: two in flight, roles alternating (no register moves)
    for (int p = wave; p < np; p += 2 * NW) {
      D1 = decode(p + NW);
      load(D1, w1);
      eval(D0, w0, p);
      D0 = decode(p + 2 * NW);
      load(D0, w0);
      eval(D1, w1, p + NW);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
      const uint32_t loc = rec[i].y;
      const int gx = wrapk(x0 - HR + (int)(loc & 31), nx), gy = wrapk(y0 - HR + (int)((loc >> 5) & 31), ny);
      const int gz = z0 - HR + (int)((loc >> 10) & 63);
      const size_t g = (size_t)gz * plane + (size_t)gy * pitch + gx;
      const T sc = scale[p0 + i];
#pragma unroll
      for (int c = 0; c < SC; ++c)
        if (s0 + c < nshots) {
          const T v = mul_rn(sc, res[c][i]);
          unew[(size_t)(s0 + c) * vol + g] += v;
          if (dd) dd[(size_t)(s0 + c) * vol + g] += v;
        }
    }
    __syncthreads();
  }
}

// The IB patch of the tiled points (column-run records), with in front of the tiles: the
// points of wider supports (nwb workgroups, one point per wavefront, the gather of k_patch;
// started first, their longer latency hides under the tiles), then the workgroups of io.
template <typename T, int SC>
__launch_bounds__(512)
__global__ void k_patch_cols(const T *__restrict__ un, T *__restrict__ unew, T *__restrict__ dd,
                             const T *__restrict__ wcol, const uint2 *__restrict__ recs, const T *__restrict__ scale,
                             const int16_t *__restrict__ zfirst, const int32_t *__restrict__ coltab,
                             const int4 *__restrict__ tiles, int ntiles, int nx, int ny, int nz, int64_t pitch,
                             int64_t vol, int nshots, const uint32_t *__restrict__ wrec, const PInfo<T> *__restrict__ wpinfo,
                             const int32_t *__restrict__ ball, const int32_t *__restrict__ wdelta,
                             const int32_t *__restrict__ ball_meta, int64_t nwide, int nwb, PatchIo<T> io) {
  const int b = (int)blockIdx.x, nsp = nwb + io.nsb + io.ninj;
  if (b < nwb) {
    const int64_t i = (int64_t)b * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (i < nwide) gather_point<T>(i, un, unew, dd, wrec, wpinfo, ball, wdelta, ball_meta, nx, ny, pitch, vol, nshots);
  } else if (b < nwb + io.nsb) {
    sample_block(un, io, b - nwb, vol);
    finish_io(io);
  } else if (b < nsp) {
    inject_sources(unew, dd, io.sidx, io.sw, nshots, vol, io.wavelet, io.wstride, io.tcount[0]);
    finish_io(io);
  } else {
    const int64_t tb = xcd_remap(b - nsp, gridDim.x - nsp);
    if (tb < ntiles)
      patch_tile<T, SC>(tb, un, unew, dd, wcol, recs, scale, zfirst, coltab, tiles, nx, ny, nz, pitch, vol, nshots);
  }
}

template <typename T>
__global__ void k_make_pinfo_dense(const int16_t *xyz, const int32_t *first, const int32_t *count,
                                   const uint32_t *doff, const T *scale, const int32_t *perm, int64_t n,
                                   PInfoD<T> *out) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t i = perm[j];
  PInfoD<T> p;
  p.x = xyz[i * 4];
  p.y = xyz[i * 4 + 1];
  p.z = xyz[i * 4 + 2];
  p.code = xyz[i * 4 + 3];
  p.first = (uint16_t)first[i];
  p.count = (uint16_t)count[i];
  p.woff = doff[i];
  p.scale = scale[i];
  out[j] = p;
}

size_t pinfo_dense_bytes(int prec) { return prec == IB_F32 ? sizeof(PInfoD<float>) : sizeof(PInfoD<double>); }

void enqueue_make_pinfo_dense(int prec, const int16_t *xyz, const int32_t *first, const int32_t *count,
                              const uint32_t *doff, const void *scale, const int32_t *perm, int64_t n, void *out,
                              hipStream_t st) {
  if (n <= 0) return;
  dim3 g((unsigned)((n + 255) / 256)), b(256);
  if (prec == IB_F32)
    hipLaunchKernelGGL(k_make_pinfo_dense<float>, g, b, 0, st, xyz, first, count, doff, (const float *)scale, perm, n,
                       (PInfoD<float> *)out);
  else
    hipLaunchKernelGGL(k_make_pinfo_dense<double>, g, b, 0, st, xyz, first, count, doff, (const double *)scale, perm,
                       n, (PInfoD<double> *)out);
}

// ---- sources and receivers ---------------------------------------------------------
template <typename T>
__global__ void k_inject(T *unew, T *dd, const int64_t *sidx, const T *sw, int nshots, int64_t vol, const T *wavelet,
                         int64_t wstride, int64_t *tcount) {
  const int64_t t = tcount[0];
  inject_sources(unew, dd, sidx, sw, nshots, vol, wavelet, wstride, t);
  __syncthreads();
  if (threadIdx.x == 0) {
    tcount[1] = t;
    tcount[0] = t + 1;
  }
}

template <typename T>
__global__ void k_sample(const T *unew, const int64_t *ridx, const T *rw, int nrec, int nshots, int64_t vol,
                         T *traces, int64_t nsteps, const int64_t *tcount) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)nrec * nshots) return;
  sample_receiver(unew, ridx, rw, nrec, vol, traces, nsteps, tcount[1] - tcount[2], e);
}

// Source injection and receiver sampling in one workgroup, for few receivers: the
// workgroup barrier orders the injection before the sampling, so the step needs one launch
// less (a small 2D step is launch-bound).  Same arithmetic as k_inject then k_sample.
template <typename T>
__global__ void k_io_small(T *unew, T *dd, const int64_t *sidx, const T *sw, int nshots, int64_t vol, const T *wavelet,
                           int64_t wstride, const int64_t *ridx, const T *rw, int nrec, T *traces, int64_t nsteps,
                           int64_t *tcount) {
  const int64_t t = tcount[0];
  for (int e = threadIdx.x; e < nshots * 8; e += blockDim.x) {
    int s = e >> 3;
    int64_t idx = sidx[e];
    if (idx >= 0) {
      const T v = mul_rn(wavelet[(size_t)s * wstride + t], sw[e]);
      unew[(size_t)s * vol + idx] += v;
      if (dd) dd[(size_t)s * vol + idx] += v;
    }
  }
  __syncthreads();
  const int64_t tl = t - tcount[2];
  for (int e = threadIdx.x; e < nrec * nshots; e += blockDim.x) {
    const int s = e / nrec, r = e % nrec;
    const T *u = unew + (size_t)s * vol;
    T v = T(0);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      int64_t idx = ridx[(size_t)r * 8 + c];
      if (idx >= 0) v += rw[(size_t)r * 8 + c] * u[idx];
    }
    traces[((size_t)s * nsteps + tl) * nrec + r] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    tcount[1] = t;
    tcount[0] = t + 1;
  }
}
constexpr int kIoSmallMax = 1024;   // receivers x shots handled by k_io_small

// Shots per pass of the tiled patch when a state holds several: each point's weights are
// loaded once for the pass, the pass's tiles of p^n sit side by side in LDS.  Two FP32 shots
// measured fastest (64 shots at 301x301x201: 92 -> 118 Gpts/s; four shots lose occupancy);
// FP64 keeps one (two FP64 tiles would leave one workgroup per CU).
template <typename T>
constexpr int kPatchShots = (sizeof(T) == 8) ? 1 : 2;
// FP32 weights are loaded in pairs (config 3 patch 0.221 -> 0.218 ms)
template <typename T>
constexpr int kPatchPairs = (sizeof(T) == 4) ? 2 : 1;

// ---- boundary values ----------------------------------------------------------------
// Inhomogeneous conditions: p^{n+1}_i += sum_q F[i][q] s_q(t_n) at every IB point, F
// holding K_i / (1 + s_i) times the point's condition-value weights contracted with g_q.
// Runs before the source injection advances the step counter.
template <typename T>
__global__ void k_ib_forcing(T *unew, T *dd, const int16_t *xyz, const T *F, const T *fs, int nq, int64_t fstride,
                             int64_t nib, int ny, int64_t pitch, int64_t vol, int nshots, const int64_t *tcount) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nib) return;
  const int64_t t = tcount[0];
  T v = T(0);
  for (int q = 0; q < nq; ++q) v += F[i * nq + q] * fs[(size_t)q * fstride + t];
  const int64_t idx = ((int64_t)xyz[i * 4 + 2] * ny + xyz[i * 4 + 1]) * pitch + xyz[i * 4];
  for (int s = 0; s < nshots; ++s) {
    unew[(size_t)s * vol + idx] += v;
    if (dd) dd[(size_t)s * vol + idx] += v;
  }
}

// ---- launch helpers ----------------------------------------------------------------
template <typename T>
static StencilW<T> stencil_weights(int M) {
  double w[2 * kMaxOrder + 1];
  second_derivative_weights(M, w);
  StencilW<T> W{};
  for (int k = 0; k <= M / 2; ++k) W.w[k] = (T)w[M / 2 + k];
  return W;
}

template <typename T, bool DL>
static void launch_interior_t(const StepArgs &a, hipStream_t st) {
  const T *un = (const T *)a.un;
  T *um = (T *)a.um;
  T *dd = (T *)a.dd;
  const T *K = (const T *)a.K;
  const T *sx = (const T *)a.sx, *sy = (const T *)a.sy, *sz = (const T *)a.sz;
  if (a.ndim == 3 && a.M == 8 && a.variant >= 1 && a.vol * (int64_t)sizeof(T) < (int64_t(1) << 31) && a.zrange16 &&
      a.zrange32) {
    const int RY = (a.variant == 2) ? 8 : (a.variant == 4 ? 2 : 4);
    const int NW = (a.variant == 3 || a.variant == 4) ? 8 : 4;
    const int TY = RY * NW;
    const int ntx = (a.nx + 63) / 64, nty = (a.ny + TY - 1) / TY;
    const int2 *zr = (TY == 32) ? a.zrange32 : a.zrange16;
    const int zc = a.zchunk > 0 ? a.zchunk : a.nz;
    const int nzc = (a.nz + zc - 1) / zc;
    int64_t nblk = (int64_t)ntx * nty * nzc * a.nshots;
    int64_t nblk8 = (nblk + 7) / 8 * 8;
    const StencilW<T> W = stencil_weights<T>(a.M);
    const StencilW<double> WD = stencil_weights<double>(a.M);
    if (a.variant == 2)
      hipLaunchKernelGGL((k_interior3d_p<T, 4, 8, 4, DL>), dim3((unsigned)nblk8), dim3(256), 0, st, un, um, dd, K, sx,
                         sy, sz, W, WD, a.nx, a.ny, a.nz, a.pitch, a.vol, zc, ntx, nty, nzc, a.nshots, zr);
    else if (a.variant == 3)
      hipLaunchKernelGGL((k_interior3d_p<T, 4, 4, 8, DL>), dim3((unsigned)nblk8), dim3(512), 0, st, un, um, dd, K, sx,
                         sy, sz, W, WD, a.nx, a.ny, a.nz, a.pitch, a.vol, zc, ntx, nty, nzc, a.nshots, zr);
    else if (a.variant == 4)
      hipLaunchKernelGGL((k_interior3d_p<T, 4, 2, 8, DL>), dim3((unsigned)nblk8), dim3(512), 0, st, un, um, dd, K, sx,
                         sy, sz, W, WD, a.nx, a.ny, a.nz, a.pitch, a.vol, zc, ntx, nty, nzc, a.nshots, zr);
    else
      hipLaunchKernelGGL((k_interior3d_p<T, 4, 4, 4, DL>), dim3((unsigned)nblk8), dim3(256), 0, st, un, um, dd, K, sx,
                         sy, sz, W, WD, a.nx, a.ny, a.nz, a.pitch, a.vol, zc, ntx, nty, nzc, a.nshots, zr);
    return;
  }
  if (a.ndim == 3 && a.M == 8) {
    constexpr int RY = 4;
    const int ntx = (a.nx + 63) / 64, nty = (a.ny + 4 * RY - 1) / (4 * RY);
    const int zc = a.zchunk > 0 ? a.zchunk : a.nz;
    const int nzc = (a.nz + zc - 1) / zc;
    int64_t nblk = (int64_t)ntx * nty * nzc * a.nshots;
    int64_t nblk8 = (nblk + 7) / 8 * 8;
    hipLaunchKernelGGL((k_interior3d<T, 4, RY, DL>), dim3((unsigned)nblk8), dim3(256), 0, st, un, um, dd, K, sx, sy,
                       sz, stencil_weights<T>(a.M), stencil_weights<double>(a.M), a.nx, a.ny, a.nz, a.pitch, a.vol, zc,
                       ntx, nty, nzc, a.nshots);
    return;
  }
  const int zf = a.zlast > a.zfirst ? a.zfirst : 0, zl = a.zlast > a.zfirst ? a.zlast : a.nz;
  const int64_t tot = (int64_t)a.nx * a.ny * (zl - zf) * a.nshots;
  if (tot == 0) return;
  dim3 g((unsigned)((tot + 255) / 256)), b(256);
  const int lat = a.ndim - 1;
  switch (a.M) {
    case 2:
      hipLaunchKernelGGL((k_interior_generic<T, 1, DL>), g, b, 0, st, un, um, dd, K, sx, sy, sz, stencil_weights<T>(2),
                         stencil_weights<double>(2), a.nx, a.ny, a.nz, lat, a.pitch, a.vol, a.nshots, zf, zl);
      break;
    case 4:
      hipLaunchKernelGGL((k_interior_generic<T, 2, DL>), g, b, 0, st, un, um, dd, K, sx, sy, sz, stencil_weights<T>(4),
                         stencil_weights<double>(4), a.nx, a.ny, a.nz, lat, a.pitch, a.vol, a.nshots, zf, zl);
      break;
    case 6:
      hipLaunchKernelGGL((k_interior_generic<T, 3, DL>), g, b, 0, st, un, um, dd, K, sx, sy, sz, stencil_weights<T>(6),
                         stencil_weights<double>(6), a.nx, a.ny, a.nz, lat, a.pitch, a.vol, a.nshots, zf, zl);
      break;
    default:
      hipLaunchKernelGGL((k_interior_generic<T, 4, DL>), g, b, 0, st, un, um, dd, K, sx, sy, sz, stencil_weights<T>(8),
                         stencil_weights<double>(8), a.nx, a.ny, a.nz, lat, a.pitch, a.vol, a.nshots, zf, zl);
      break;
  }
}

template <typename T>
static void launch_interior(const StepArgs &a, hipStream_t st) {
  if (a.dd)
    launch_interior_t<T, true>(a, st);
  else
    launch_interior_t<T, false>(a, st);
}

template <typename T>
static void launch_patch(const StepArgs &a, hipStream_t st, const PatchIo<T> *io_in = nullptr) {
  // the column-run kernels take the wide points in their first workgroups; the other
  // layouts leave them to the gather kernel, on the second stream beside them
  const bool merged = a.ntiles > 0 && (a.patch_variant == 8 || a.patch_variant == 9);
  const int nwb = merged ? (int)((a.nwide + 7) / 8) : 0;
  if (!merged && a.ntiles > 0 && a.nwide > 0 && a.aux != nullptr) (void)hipEventRecord(a.ev_fork, st);
  if (a.ntiles > 0) {
    int64_t nblk = ((int64_t)a.ntiles + 7) / 8 * 8;
#define IB_PATCH_TILED(PVV)                                                                                         \
  hipLaunchKernelGGL((k_patch_tiled<T, kTileX, kTileY, kTileZ, kTileHalo, PVV>), dim3((unsigned)nblk), dim3(512), 0, \
                     st, (const T *)a.un, (T *)a.um, (T *)a.dd, (const T *)a.dense, (const PInfoD<T> *)a.pinfo, a.ball, \
                     a.ball_meta, a.tiles, a.ntiles, a.nx, a.ny, a.nz, a.pitch, a.vol, a.nshots)
#define IB_PATCH_TILED_R(DD, SC)                                                                                    \
  hipLaunchKernelGGL((k_patch_tiled_r<T, kTileX, kTileY, kTileZ, kTileHalo, DD, SC, kPatchPairs<T>>),                  \
                     dim3((unsigned)nblk),                                                                           \
                     dim3(512),                                                                                      \
                     0, st, (const T *)a.un, (T *)a.um, (T *)a.dd, (const T *)a.dense, (const PInfoD<T> *)a.pinfo,    \
                     a.ball, a.ball_meta, a.tiles, a.ntiles, a.nx, a.ny, a.nz, a.pitch, a.vol, a.nshots)
    switch (a.patch_variant) {
      case 0: IB_PATCH_TILED(0); break;
      case 1: IB_PATCH_TILED(1); break;
      case 2: IB_PATCH_TILED(2); break;
      case 3: IB_PATCH_TILED(3); break;
      case 4:
        if (a.nshots >= kPatchShots<T>)
          IB_PATCH_TILED_R(1, kPatchShots<T>);
        else
          IB_PATCH_TILED_R(1, 1);
        break;
      case 5: IB_PATCH_TILED_R(2, 1); break;
      case 6: IB_PATCH_TILED_R(3, 1); break;
      case 8:
      case 9: {
        // two shots per pass in FP32 only (two FP64 tiles would not leave room for a second
        // workgroup per CU)
        bool two = false;
        PatchIo<T> io = io_in ? *io_in : PatchIo<T>{};
        io.nsb = (int)std::min<int64_t>((io.nrs + 511) / 512, kMaxSampleBlocks);
        const unsigned grid = (unsigned)(nblk + nwb + io.nsb + io.ninj);
        if constexpr (sizeof(T) == 4) {
          two = a.patch_variant == 9 && a.nshots >= 2;
          if (two)
            hipLaunchKernelGGL((k_patch_cols<T, 2>), dim3(grid), dim3(512), 0, st, (const T *)a.un, (T *)a.um,
                               (T *)a.dd, (const T *)a.wcol, a.crec, (const T *)a.cscale, a.zfcol, a.coltab, a.tiles,
                               a.ntiles, a.nx, a.ny, a.nz, a.pitch, a.vol, a.nshots, a.rec, (const PInfo<T> *)a.pinfo_wide,
                               a.ball, a.delta, a.ball_meta, a.nwide, nwb, io);
        }
        if (!two)
          hipLaunchKernelGGL((k_patch_cols<T, 1>), dim3(grid), dim3(512), 0, st, (const T *)a.un, (T *)a.um,
                             (T *)a.dd, (const T *)a.wcol, a.crec, (const T *)a.cscale, a.zfcol, a.coltab, a.tiles,
                             a.ntiles, a.nx, a.ny, a.nz, a.pitch, a.vol, a.nshots, a.rec, (const PInfo<T> *)a.pinfo_wide,
                             a.ball, a.delta, a.ball_meta, a.nwide, nwb, io);
        break;
      }
      default:
        hipLaunchKernelGGL((k_patch_tiled_m<T, kTileX, kTileY, kTileZ, kTileHalo>), dim3((unsigned)nblk), dim3(512), 0,
                           st, (const T *)a.un, (T *)a.um, (T *)a.dd, a.rec, (const PInfo<T> *)a.pinfo_tm, a.ball,
                           a.ball_meta,
                           a.tiles, a.ntiles, a.nx, a.ny, a.nz, a.pitch, a.vol, a.nshots);
        break;
    }
#undef IB_PATCH_TILED
#undef IB_PATCH_TILED_R
  }
  if (a.nwide > 0 && !merged) {
    // the few points with wider supports touch other nodes than the tiled points: their
    // gather kernel runs on the second stream, beside the tiled kernel
    const bool fork = a.ntiles > 0 && a.aux != nullptr;
    hipStream_t ws = fork ? a.aux : st;
    if (fork) (void)hipStreamWaitEvent(a.aux, a.ev_fork, 0);
    int64_t nblk = ((a.nwide + 3) / 4 + 7) / 8 * 8;
    PatchIo<T> io = (io_in && !fork) ? *io_in : PatchIo<T>{};
    io.nsb = (int)std::min<int64_t>((io.nrs + 255) / 256, kMaxSampleBlocks);
    hipLaunchKernelGGL(k_patch<T>, dim3((unsigned)(nblk + io.nsb + io.ninj)), dim3(256), 0, ws, (const T *)a.un,
                       (T *)a.um, (T *)a.dd, a.rec, (const PInfo<T> *)a.pinfo_wide, a.ball, a.delta, a.ball_meta,
                       a.nwide, a.nx, a.ny, a.nz, a.pitch, a.vol, a.nshots, io);
    if (fork) {
      (void)hipEventRecord(a.ev_join, a.aux);
      (void)hipStreamWaitEvent(st, a.ev_join, 0);
    }
  }
}

template <typename T>
static void launch_io(const StepArgs &a, T *u, hipStream_t st) {
  if (a.nrec > 0 && a.traces && (int64_t)a.nrec * a.nshots <= kIoSmallMax) {
    hipLaunchKernelGGL(k_io_small<T>, dim3(1), dim3(256), 0, st, u, (T *)a.dd, a.sidx, (const T *)a.sw, a.nshots, a.vol,
                       (const T *)a.wavelet, a.wstride, a.ridx, (const T *)a.rw, a.nrec, (T *)a.traces, a.nsteps,
                       a.tcount);
    return;
  }
  hipLaunchKernelGGL(k_inject<T>, dim3(1), dim3(256), 0, st, u, (T *)a.dd, a.sidx, (const T *)a.sw, a.nshots, a.vol,
                     (const T *)a.wavelet, a.wstride, a.tcount);
  if (a.nrec > 0 && a.traces) {
    int64_t tot = (int64_t)a.nrec * a.nshots;
    hipLaunchKernelGGL(k_sample<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, (const T *)u, a.ridx,
                       (const T *)a.rw, a.nrec, a.nshots, a.vol, (T *)a.traces, a.nsteps, (const int64_t *)a.tcount);
  }
}

// whether the step's source injection and sampling ride in the column-run patch launch
static bool io_in_patch(const StepArgs &a) {
  if (!a.io_merge || a.fF) return false;
  if (a.ntiles > 0) return a.ndim == 3 && (a.patch_variant == 8 || a.patch_variant == 9);
  return a.nwide > 0;   // the gather patch alone (2D)
}

template <typename T>
static void launch_step(const StepArgs &a, hipStream_t st) {
  launch_interior<T>(a, st);
  if (io_in_patch(a)) {
    PatchIo<T> io{};
    if (a.sample_prev && a.nrec > 0 && a.traces) {
      io.ridx = a.ridx;
      io.rw = (const T *)a.rw;
      io.nrec = a.nrec;
      io.nrs = (int64_t)a.nrec * a.nshots;
      io.traces = (T *)a.traces;
      io.nsteps = a.nsteps;
    }
    io.sidx = a.sidx;
    io.sw = (const T *)a.sw;
    io.wavelet = (const T *)a.wavelet;
    io.wstride = a.wstride;
    io.ninj = 1;
    io.tcount = a.tcount;
    io.advance = 1;
    launch_patch<T>(a, st, &io);
    return;
  }
  launch_patch<T>(a, st);
  if (a.fF && a.nib > 0)
    hipLaunchKernelGGL(k_ib_forcing<T>, dim3((unsigned)((a.nib + 255) / 256)), dim3(256), 0, st, (T *)a.um,
                       (T *)a.dd, a.ib_xyz,
                       (const T *)a.fF, (const T *)a.fs, a.fnq, a.fstride, a.nib, a.ny, a.pitch, a.vol, a.nshots,
                       (const int64_t *)a.tcount);
  launch_io<T>(a, (T *)a.um, st);
}

void enqueue_source_receivers(const StepArgs &a, void *u, hipStream_t st) {
  if (a.prec == IB_F32)
    launch_io<float>(a, (float *)u, st);
  else
    launch_io<double>(a, (double *)u, st);
}

template <typename T>
static void launch_sample(const StepArgs &a, const T *u, hipStream_t st) {
  if (!(a.nrec > 0 && a.traces)) return;
  const int64_t tot = (int64_t)a.nrec * a.nshots;
  hipLaunchKernelGGL(k_sample<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, u, a.ridx, (const T *)a.rw,
                     a.nrec, a.nshots, a.vol, (T *)a.traces, a.nsteps, (const int64_t *)a.tcount);
}

void enqueue_sample(const StepArgs &a, const void *u, hipStream_t st) {
  if (a.prec == IB_F32)
    launch_sample<float>(a, (const float *)u, st);
  else
    launch_sample<double>(a, (const double *)u, st);
}

bool step_samples_in_patch(const StepArgs &a) { return io_in_patch(a); }

void enqueue_step(const StepArgs &a, hipStream_t st) {
  if (a.prec == IB_F32)
    launch_step<float>(a, st);
  else
    launch_step<double>(a, st);
}

void enqueue_interior_only(const StepArgs &a, hipStream_t st) {
  if (a.prec == IB_F32)
    launch_interior<float>(a, st);
  else
    launch_interior<double>(a, st);
}

void enqueue_patch_only(const StepArgs &a, hipStream_t st) {
  if (a.prec == IB_F32)
    launch_patch<float>(a, st);
  else
    launch_patch<double>(a, st);
}

// ---- discrete adjoint ----------------------------------------------------------------
// With D = 1/(1+s), the adjoint of the damped leapfrog (scaled lambda = D mu') is the same
// recurrence with L^T K in place of K L:
//   lambda^m = D [2 lambda^{m+1} - (1 - s) lambda^{m+2} + L^T (K lambda^{m+1}) + R^T res^{m-1}],
// and dJ/dK = sum_m lambda^m (L u^{m-1}).  The adjoint runs on mu = K lambda: multiplying by
// K gives mu^m = D [2 mu^{m+1} - (1 - s) mu^{m+2} + K L_std(mu^{m+1})] + K D (IB^T mu^{m+1} +
// R^T res^{m-1}), because the standard stencil is symmetric.  The first part is the forward
// interior kernel applied to mu; the IB rows are transposed through a per-receiving-node
// table (a gather, deterministic, no atomics) and the receivers likewise, both with the
// factor K_j D_j.  (lambda and mu differ only where K = 0, where lambda never feeds back.)
// The gradient needs L u^{m-1} with the IB rows; the forward step gives it pointwise:
//   K L u^{m-1} = (1 + s) u^m - 2 u^{m-1} + (1 - s) u^{m-2} - (1 + s) (source injected into u^m),
// so with lambda = mu / K, dJ/dK = (sum_m mu^m (K L u^{m-1})) / K^2: the sum is accumulated
// in FP64 and divided once at the end.

// v[i][s] = mu^{m+1}_{s,i} at the IB points (shots fastest), for the gather below
template <typename T>
__global__ void k_adj_ibvals(T *__restrict__ v, const T *__restrict__ lam1, const int16_t *__restrict__ xyz,
                             int64_t nib, int nshots, int ny, int64_t pitch, int64_t vol) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nib * nshots) return;
  const int64_t i = e / nshots;
  const int s = (int)(e - i * nshots);
  const size_t q = ((size_t)xyz[i * 4 + 2] * ny + xyz[i * 4 + 1]) * pitch + xyz[i * 4];
  v[e] = lam1[(size_t)s * vol + q];
}

// mu^m_j += (K D)_j sum_k w_k v[i_k] over the IB points i_k whose rows use node j, for SC
// shots at a time.  A 16-lane row of a wavefront takes one receiving node: its lanes read
// the node's run of (point, weight) entries together (coalesced), gather v, and the row's
// partial sums are combined with DPP rotations inside the row.
template <typename T, int SC>
__launch_bounds__(256)
__global__ void k_adj_gather(T *__restrict__ lam, T *__restrict__ lamd, const T *__restrict__ v,
                             const uint32_t *__restrict__ jnode,
                             const T *__restrict__ jD, const uint32_t *__restrict__ joff,
                             const uint32_t *__restrict__ src, const T *__restrict__ wt, int64_t nj, int nshots,
                             int s0, int64_t vol) {
  const int sub = threadIdx.x & 15;
  const int64_t j = (int64_t)blockIdx.x * (blockDim.x >> 4) + (threadIdx.x >> 4);
  const bool live = j < nj;
  // rows stay complete (no early return) so that the DPP rotations see all 16 lanes
  const uint32_t a = live ? joff[j] : 0u, b = live ? joff[j + 1] : 0u;
  T acc[SC];
#pragma unroll
  for (int c = 0; c < SC; ++c) acc[c] = T(0);
  // a point's SC values as 16-byte loads where they are aligned to them (the same products
  // and sums as the element loads)
  constexpr int VW = 16 / sizeof(T);
  if (SC % VW == 0 && nshots % VW == 0 && s0 % VW == 0 && s0 + SC <= nshots) {
    for (uint32_t k = a + sub; k < b; k += 16) {
      const T w = wt[k];
      const T *vi = v + (size_t)src[k] * nshots + s0;
#pragma unroll
      for (int c = 0; c < SC; c += VW) {
        T q[VW];
        __builtin_memcpy(q, __builtin_assume_aligned(vi + c, 16), 16);
#pragma unroll
        for (int e = 0; e < VW; ++e) acc[c + e] += w * q[e];
      }
    }
  } else {
    for (uint32_t k = a + sub; k < b; k += 16) {
      const T w = wt[k];
      const T *vi = v + (size_t)src[k] * nshots + s0;
#pragma unroll
      for (int c = 0; c < SC; ++c)
        if (s0 + c < nshots) acc[c] += w * vi[c];
    }
  }
  T mine = T(0);
#pragma unroll
  for (int c = 0; c < SC; ++c) {
    const T t = row_sum16(acc[c]);
    if (sub == c) mine = t;
  }
  if (live && sub < SC && s0 + sub < nshots) {
    const size_t g = (size_t)(s0 + sub) * vol + jnode[j];
    const T add = mul_rn(jD[j], mine);
    lam[g] += add;
    if (lamd) lamd[g] += add;
  }
}

// mu^m_j += (K D)_j sum over receivers using node j of w * res^{m-1}
template <typename T>
__global__ void k_adj_receivers(T *__restrict__ lam, T *__restrict__ lamd, const T *__restrict__ res, int64_t nt,
                                int nrec, int64_t step,
                                const int64_t *__restrict__ rnode, const T *__restrict__ rD,
                                const int64_t *__restrict__ roff, const int32_t *__restrict__ rrec,
                                const T *__restrict__ rw, int64_t nrn, int nshots, int64_t vol) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrn) return;
  const int64_t a = roff[j], b = roff[j + 1];
  for (int s = 0; s < nshots; ++s) {
    const T *r = res + ((size_t)s * nt + step) * nrec;
    T acc = T(0);
    for (int64_t k = a; k < b; ++k) acc += rw[k] * r[rrec[k]];
    const size_t g = (size_t)s * vol + rnode[j];
    const T add = mul_rn(rD[j], acc);
    lam[g] += add;
    if (lamd) lamd[g] += add;
  }
}

// g += sum over shots of mu^m ((1 + s) u^m - 2 u^{m-1} + (1 - s) u^{m-2}) at interior nodes,
// in FP64 from the stored time levels; one thread per node of a padded row.  In the
// increment form the segment keeps d^m = u^m - u^{m-1} and the same quantity is
// (1 + s) d^m - (1 - s) d^{m-1} (u1 is null, u2 = d^m, u0 = d^{m-1}).
template <typename T>
__launch_bounds__(256)
__global__ void k_grad_pt(double *__restrict__ gK, const T *__restrict__ mu, const T *__restrict__ u2,
                          const T *__restrict__ u1, const T *__restrict__ u0, const T *__restrict__ K,
                          const T *__restrict__ sx, const T *__restrict__ sy, const T *__restrict__ sz, int nx,
                          int ny, int64_t pitch, int64_t vol, int nshots) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  if (x >= nx) return;
  const size_t c = ((size_t)z * ny + y) * pitch + x;
  if (K[c] == T(0)) return;
  const double s = (double)sx[x] + (double)sy[y] + (double)sz[z];
  double tot = 0.0;
  for (int sh = 0; sh < nshots; ++sh) {
    const size_t q = (size_t)sh * vol + c;
    // the time levels are read once here: non-temporal
    double l;
    if (u1)
      l = (1.0 + s) * (double)__builtin_nontemporal_load(&u2[q]) - 2.0 * (double)__builtin_nontemporal_load(&u1[q]) +
          (1.0 - s) * (double)__builtin_nontemporal_load(&u0[q]);
    else
      l = (1.0 + s) * (double)__builtin_nontemporal_load(&u2[q]) - (1.0 - s) * (double)__builtin_nontemporal_load(&u0[q]);
    tot += (double)mu[q] * l;
  }
  gK[c] += tot;
}

// the source injected into u^m is not part of K L u^{m-1}: remove its term (one thread, in
// order, so the accumulation stays deterministic)
template <typename T>
__global__ void k_grad_src(double *__restrict__ gK, const T *__restrict__ mu, const int64_t *__restrict__ sidx,
                           const T *__restrict__ sw, const T *__restrict__ wavelet, int64_t wstride, int64_t t,
                           const T *__restrict__ sx, const T *__restrict__ sy, const T *__restrict__ sz, int ny,
                           int64_t pitch, int64_t vol, int nshots) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  for (int e = 0; e < nshots * 8; ++e) {
    const int64_t q = sidx[e];
    if (q < 0) continue;
    const int sh = e >> 3;
    const int x = (int)(q % pitch);
    const int64_t r = q / pitch;
    const int y = (int)(r % ny), z = (int)(r / ny);
    const double s = (double)sx[x] + (double)sy[y] + (double)sz[z];
    const double inj = (double)(wavelet[(size_t)sh * wstride + t] * sw[e]);
    gK[q] -= (double)mu[(size_t)sh * vol + q] * (1.0 + s) * inj;
  }
}

template <typename T>
__global__ void k_grad_out(const double *__restrict__ gK, const T *__restrict__ K, double *__restrict__ out, int nx,
                           int ny, int nz, int64_t pitch, double dt_over_h) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t per = (int64_t)nx * ny * nz;
  if (i >= per) return;
  const int x = (int)(i % nx);
  int64_t r = i / nx;
  const int y = (int)(r % ny);
  const int z = (int)(r / ny);
  const size_t c = ((size_t)z * ny + y) * pitch + x;
  const double k = (double)K[c];
  // gK holds sum mu (K L u) = K^2 dJ/dK; dK/dc = 2 sqrt(K) dt / h
  out[i] = (k > 0.0) ? gK[c] / (k * k) * 2.0 * sqrt(k) * dt_over_h : 0.0;
}

template <typename T>
static void adjoint_step_t(const AdjArgs &a, hipStream_t st) {
  if (a.nj > 0) {
    const int64_t nv = a.nib * a.nshots;
    hipLaunchKernelGGL(k_adj_ibvals<T>, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, st, (T *)a.vals,
                       (const T *)a.lam1, a.ibxyz, a.nib, a.nshots, a.ny, a.pitch, a.vol);
    const dim3 gj((unsigned)((a.nj + 15) / 16));
    for (int s0 = 0; s0 < a.nshots;) {
      const int left = a.nshots - s0;
      if (left >= 16) {
        hipLaunchKernelGGL((k_adj_gather<T, 16>), gj, dim3(256), 0, st, (T *)a.lam2, (T *)a.lamd, (const T *)a.vals,
                           a.jnode,
                           (const T *)a.jD, a.joff, a.jsrc, (const T *)a.jw, a.nj, a.nshots, s0, a.vol);
        s0 += 16;
      } else if (left >= 8) {
        hipLaunchKernelGGL((k_adj_gather<T, 8>), gj, dim3(256), 0, st, (T *)a.lam2, (T *)a.lamd, (const T *)a.vals,
                           a.jnode,
                           (const T *)a.jD, a.joff, a.jsrc, (const T *)a.jw, a.nj, a.nshots, s0, a.vol);
        s0 += 8;
      } else if (left >= 4) {
        hipLaunchKernelGGL((k_adj_gather<T, 4>), gj, dim3(256), 0, st, (T *)a.lam2, (T *)a.lamd, (const T *)a.vals,
                           a.jnode,
                           (const T *)a.jD, a.joff, a.jsrc, (const T *)a.jw, a.nj, a.nshots, s0, a.vol);
        s0 += 4;
      } else {
        hipLaunchKernelGGL((k_adj_gather<T, 1>), gj, dim3(256), 0, st, (T *)a.lam2, (T *)a.lamd, (const T *)a.vals,
                           a.jnode,
                           (const T *)a.jD, a.joff, a.jsrc, (const T *)a.jw, a.nj, a.nshots, s0, a.vol);
        s0 += 1;
      }
    }
  }
  if (a.nrn > 0)
    hipLaunchKernelGGL(k_adj_receivers<T>, dim3((unsigned)((a.nrn + 255) / 256)), dim3(256), 0, st, (T *)a.lam2,
                       (T *)a.lamd, (const T *)a.res, a.nt, a.nrec, a.step, a.rnode, (const T *)a.rD, a.roff, a.rrec,
                       (const T *)a.rw, a.nrn, a.nshots, a.vol);
  const dim3 gg((unsigned)((a.nx + 255) / 256), (unsigned)a.ny, (unsigned)a.nz);
  hipLaunchKernelGGL(k_grad_pt<T>, gg, dim3(256), 0, st, a.gK, (const T *)a.lam2, (const T *)a.u2,
                     (const T *)a.u1, (const T *)a.u0, (const T *)a.K, (const T *)a.sx, (const T *)a.sy,
                     (const T *)a.sz, a.nx, a.ny, a.pitch, a.vol, a.nshots);
  hipLaunchKernelGGL(k_grad_src<T>, dim3(1), dim3(64), 0, st, a.gK, (const T *)a.lam2, a.sidx, (const T *)a.sw,
                     (const T *)a.wavelet, a.wstride, a.step, (const T *)a.sx, (const T *)a.sy, (const T *)a.sz, a.ny,
                     a.pitch, a.vol, a.nshots);
}

void enqueue_adjoint_step(const AdjArgs &a, hipStream_t st) {
  if (a.prec == IB_F32)
    adjoint_step_t<float>(a, st);
  else
    adjoint_step_t<double>(a, st);
}

void enqueue_grad_out(int prec, const double *gK, const void *K, double *out, int nx, int ny, int nz, int64_t pitch,
                      double dt_over_h, hipStream_t st) {
  int64_t per = (int64_t)nx * ny * nz;
  dim3 g((unsigned)((per + 255) / 256)), b(256);
  if (prec == IB_F32)
    hipLaunchKernelGGL(k_grad_out<float>, g, b, 0, st, gK, (const float *)K, out, nx, ny, nz, pitch, dt_over_h);
  else
    hipLaunchKernelGGL(k_grad_out<double>, g, b, 0, st, gK, (const double *)K, out, nx, ny, nz, pitch, dt_over_h);
}

size_t pinfo_bytes(int prec) { return prec == IB_F32 ? sizeof(PInfo<float>) : sizeof(PInfo<double>); }

// per-point records and per-layout offset tables of a state
template <typename T>
__global__ void k_make_pinfo(const int16_t *xyz, const uint32_t *roff, const T *scale, const int32_t *perm,
                             int64_t nib, PInfo<T> *out) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nib) return;
  const int64_t i = perm ? perm[j] : j;
  PInfo<T> p;
  p.x = xyz[i * 4];
  p.y = xyz[i * 4 + 1];
  p.z = xyz[i * 4 + 2];
  p.code = xyz[i * 4 + 3];
  p.roff = roff[i];
  p.pad = 0;
  p.scale = scale[i];
  out[j] = p;
}

__global__ void k_make_delta(const int32_t *ball, int n, int64_t pitch, int64_t plane, int32_t *delta) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t v = (uint32_t)ball[i];
  int dx = (int8_t)(v & 255), dy = (int8_t)((v >> 8) & 255), dz = (int8_t)((v >> 16) & 255);
  delta[i] = (int32_t)(dz * plane + dy * pitch + dx);
}

void enqueue_make_pinfo(int prec, const int16_t *xyz, const uint32_t *roff, const void *scale, const int32_t *perm,
                        int64_t n, void *out, hipStream_t st) {
  if (n <= 0) return;
  if (prec == IB_F32)
    hipLaunchKernelGGL(k_make_pinfo<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, xyz, roff,
                       (const float *)scale, perm, n, (PInfo<float> *)out);
  else
    hipLaunchKernelGGL(k_make_pinfo<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, xyz, roff,
                       (const double *)scale, perm, n, (PInfo<double> *)out);
}

void enqueue_make_delta(const int32_t *ball, int n, int64_t pitch, int64_t plane, int32_t *delta, hipStream_t st) {
  hipLaunchKernelGGL(k_make_delta, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ball, n, pitch, plane, delta);
}

}  // namespace ib
