// Transposed immersed-boundary rows for the discrete adjoint, built on the GPU.
//
// The adjoint of the stepper applies L^T to K lambda (see step.hip).  The IB part of L^T
// sends the extrapolation weight y_ij of IB point i and data node j from row i to row j,
// so each receiving node j gathers sum_i y_ij (K lambda)_i over the IB points whose
// supports use it.  The table (receiving nodes, per-node runs of (IB point, weight)) is
// built once per stencil table: one wavefront per IB point emits its (node, entry) pairs
// from the data-membership masks, a radix sort by receiving node groups them (stable, so
// each run lists its IB points in ascending order and the sums are deterministic), and a
// run-length encoding gives the run offsets.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>

#include "ib_internal.h"
#include "step.h"

namespace ib {

namespace {

__device__ __forceinline__ int wrapq(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// one wavefront per IB point: key = padded index of each data node of its support,
// pt = the point, at the point's weight positions (w64 order)
__global__ void k_adj_entries(const int16_t *__restrict__ xyz, const int32_t *__restrict__ meta,
                              const uint32_t *__restrict__ rec32, const uint32_t *__restrict__ roff32,
                              const int32_t *__restrict__ ball, const int32_t *__restrict__ ball_meta, int64_t nib,
                              int nx, int ny, int64_t pitch, uint32_t *__restrict__ key, uint32_t *__restrict__ pt,
                              uint32_t *__restrict__ idx) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= nib) return;
  const int x = xyz[i * 4], y = xyz[i * 4 + 1], z = xyz[i * 4 + 2], code = xyz[i * 4 + 3];
  const int st0 = ball_meta[2 * code], nb = ball_meta[2 * code + 1];
  const uint32_t *m = rec32 + roff32[i];
  int64_t e = meta[i * 4 + 3];
  for (int b0 = 0; b0 < nb; b0 += 64) {
    const int b = b0 + lane;
    const bool on = b < nb && ((m[b >> 5] >> (b & 31)) & 1u);
    const uint64_t bal = __ballot(on);
    if (on) {
      const int rank = __popcll(bal & ((1ull << lane) - 1ull));
      const uint32_t v = (uint32_t)ball[st0 + b];
      const int dx = (int8_t)(v & 255), dy = (int8_t)((v >> 8) & 255), dz = (int8_t)((v >> 16) & 255);
      const int xx = wrapq(x + dx, nx), yy = wrapq(y + dy, ny), zz = z + dz;
      key[e + rank] = (uint32_t)(((int64_t)zz * ny + yy) * pitch + xx);
      pt[e + rank] = (uint32_t)i;
      idx[e + rank] = (uint32_t)(e + rank);
    }
    e += __popcll(bal);
  }
}

template <typename T>
__global__ void k_adj_fill(const uint32_t *__restrict__ sorted_idx, const uint32_t *__restrict__ pt,
                           const double *__restrict__ w64, int64_t n, uint32_t *__restrict__ jsrc,
                           T *__restrict__ jw) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint32_t e = sorted_idx[k];
  jsrc[k] = pt[e];
  jw[k] = (T)w64[e];
}

__global__ void k_adj_offsets(const uint32_t *__restrict__ counts, const uint32_t *__restrict__ excl,
                              const int *__restrict__ nruns, uint32_t *__restrict__ joff) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int n = *nruns;
  if (r < n) joff[r] = excl[r];
  if (r == n - 1) joff[n] = excl[r] + counts[r];
}

}  // namespace

ib_status adjoint_table_build(ib_weights *w, hipStream_t st) {
  if (w->adj_nj >= 0) return IB_OK;
  const int64_t n = w->sumw;
  const int64_t vol = w->pitch * w->ny * w->nz;
  if (vol >= (int64_t(1) << 32) || n >= (int64_t(1) << 31)) {
    set_error("adjoint table: grid or weight count exceeds 32-bit indexing");
    return IB_ERR_ARG;
  }
  ib_status s;
  if (n == 0) {
    if ((s = dalloc_t(&w->adj_joff, 1))) return s;
    IB_HIP(hipMemsetAsync(w->adj_joff, 0, 4, st));
    IB_HIP(hipStreamSynchronize(st));
    w->adj_nj = 0;
    return IB_OK;
  }
  uint32_t *key = nullptr, *key2 = nullptr, *pt = nullptr, *idx = nullptr, *idx2 = nullptr, *counts = nullptr,
           *excl = nullptr;
  int *nruns = nullptr;
  void *tmp = nullptr;
  auto cleanup = [&]() {
    dfree(key), dfree(key2), dfree(pt), dfree(idx), dfree(idx2), dfree(counts), dfree(excl), dfree(nruns), dfree(tmp);
  };
  if ((s = dalloc_t(&key, n)) || (s = dalloc_t(&key2, n)) || (s = dalloc_t(&pt, n)) || (s = dalloc_t(&idx, n)) ||
      (s = dalloc_t(&idx2, n)) || (s = dalloc_t(&nruns, 1))) {
    cleanup();
    return s;
  }
  {
    const int64_t nblk = (w->nib + 3) / 4;
    hipLaunchKernelGGL(k_adj_entries, dim3((unsigned)nblk), dim3(256), 0, st, w->ib_xyz, w->ib_meta, w->rec32,
                       w->rec_off32, w->ball, w->ball_meta, w->nib, (int)w->nx, (int)w->ny, w->pitch, key, pt, idx);
    IB_HIP(hipGetLastError());
  }
  int nbits = 1;
  while ((int64_t(1) << nbits) < vol) ++nbits;
  size_t tb_sort = 0, tb_rle = 0, tb_scan = 0;
  IB_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb_sort, key, key2, idx, idx2, (int)n, 0, nbits, st));
  IB_HIP(hipcub::DeviceRunLengthEncode::Encode(nullptr, tb_rle, key2, key, idx, nruns, (int)n, st));
  IB_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb_scan, idx, pt, (int)n, st));
  size_t tb = std::max(tb_sort, std::max(tb_rle, tb_scan));
  if ((s = dalloc(&tmp, std::max<size_t>(tb, 1)))) {
    cleanup();
    return s;
  }
  // sort (node, entry) by node; the stable radix sort keeps entries of a node in point order
  IB_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb, key, key2, idx, idx2, (int)n, 0, nbits, st));
  // per-entry IB point and weight in sorted order (pt and w64 are indexed by entry)
  if ((s = dalloc_t(&w->adj_jsrc, n)) || (s = dalloc_t(&w->adj_jw32, n)) || (s = dalloc_t(&w->adj_jw64, n))) {
    cleanup();
    return s;
  }
  {
    dim3 g((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL(k_adj_fill<float>, g, dim3(256), 0, st, idx2, pt, w->w64, n, w->adj_jsrc, w->adj_jw32);
    hipLaunchKernelGGL(k_adj_fill<double>, g, dim3(256), 0, st, idx2, pt, w->w64, n, w->adj_jsrc, w->adj_jw64);
    IB_HIP(hipGetLastError());
  }
  // runs of equal receiving nodes: unique nodes (into key), run lengths (into idx)
  IB_HIP(hipcub::DeviceRunLengthEncode::Encode(tmp, tb, key2, key, idx, nruns, (int)n, st));
  int nr = 0;
  IB_HIP(hipMemcpyAsync(&nr, nruns, sizeof(int), hipMemcpyDeviceToHost, st));
  IB_HIP(hipStreamSynchronize(st));
  counts = idx;
  idx = nullptr;
  excl = pt;
  pt = nullptr;
  IB_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, counts, excl, nr, st));
  if ((s = dalloc_t(&w->adj_jnode, std::max(nr, 1))) || (s = dalloc_t(&w->adj_joff, nr + 1))) {
    cleanup();
    return s;
  }
  IB_HIP(hipMemcpyAsync(w->adj_jnode, key, (size_t)nr * 4, hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL(k_adj_offsets, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, st, counts, excl, nruns,
                     w->adj_joff);
  IB_HIP(hipGetLastError());
  IB_HIP(hipStreamSynchronize(st));
  cleanup();
  w->adj_nj = nr;
  return IB_OK;
}

// ---- per-step kernels --------------------------------------------------------------
// D_j = 1 / (1 + s_j) at the receiving nodes (per state: the damping is the state's)
template <typename T>
__global__ void k_adj_D(const uint32_t *__restrict__ jnode, int64_t nj, const T *__restrict__ K,
                        const T *__restrict__ sx, const T *__restrict__ sy, const T *__restrict__ sz, int ny,
                        int64_t pitch, T *__restrict__ D) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nj) return;
  const int64_t q = jnode[j];
  const int x = (int)(q % pitch);
  const int64_t r = q / pitch;
  const int y = (int)(r % ny), z = (int)(r / ny);
  D[j] = K[q] / (T(1) + sx[x] + sy[y] + sz[z]);
}

// receiving-node factor K_j / (1 + s_j) of the transposed IB rows (the adjoint runs on
// mu = K lambda)
void enqueue_adj_D(int prec, const uint32_t *jnode, int64_t nj, const void *K, const void *sx, const void *sy,
                   const void *sz, int ny, int64_t pitch, void *D, hipStream_t st) {
  if (nj <= 0) return;
  dim3 g((unsigned)((nj + 255) / 256)), b(256);
  if (prec == IB_F32)
    hipLaunchKernelGGL(k_adj_D<float>, g, b, 0, st, jnode, nj, (const float *)K, (const float *)sx,
                       (const float *)sy, (const float *)sz, ny, pitch, (float *)D);
  else
    hipLaunchKernelGGL(k_adj_D<double>, g, b, 0, st, jnode, nj, (const double *)K, (const double *)sx,
                       (const double *)sy, (const double *)sz, ny, pitch, (double *)D);
}

template <typename T>
__global__ void k_scale_by_K(T *__restrict__ v, const int64_t *__restrict__ node, int64_t n, const T *__restrict__ K) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) v[j] *= K[node[j]];
}

void enqueue_scale_by_K(int prec, void *v, const int64_t *node, int64_t n, const void *K, hipStream_t st) {
  if (n <= 0) return;
  dim3 g((unsigned)((n + 255) / 256)), b(256);
  if (prec == IB_F32)
    hipLaunchKernelGGL(k_scale_by_K<float>, g, b, 0, st, (float *)v, node, n, (const float *)K);
  else
    hipLaunchKernelGGL(k_scale_by_K<double>, g, b, 0, st, (double *)v, node, n, (const double *)K);
}

}  // namespace ib
