// Device helpers shared by the step kernels: a separately rounded product, source
// injection, receiver sampling, and the io workgroups that carry them inside a patch launch.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ib {

// a product rounded on its own (never fused into a later addition): a term added to both the
// field and the increment of the increment form rounds the same in every kernel variant
template <typename T>
__device__ __forceinline__ T mul_rn(T a, T b) {
#pragma clang fp contract(off)
  return a * b;
}

// ---- sources and receivers (also run inside the patch launches) ----------------------
template <typename T>
__device__ __forceinline__ void inject_sources(T *unew, T *dd, const int64_t *sidx, const T *sw, int nshots, int64_t vol,
                                               const T *wavelet, int64_t wstride, int64_t t) {
  for (int e = threadIdx.x; e < nshots * 8; e += blockDim.x) {
    int s = e >> 3;
    int64_t idx = sidx[e];
    if (idx >= 0) {
      const T v = mul_rn(wavelet[(size_t)s * wstride + t], sw[e]);
      unew[(size_t)s * vol + idx] += v;
      if (dd) dd[(size_t)s * vol + idx] += v;
    }
  }
}

// receiver e (shot e / nrec) of field u into trace row tl
template <typename T>
__device__ __forceinline__ void sample_receiver(const T *u0, const int64_t *ridx, const T *rw, int nrec, int64_t vol,
                                                T *traces, int64_t nsteps, int64_t tl, int64_t e) {
  const int s = (int)(e / nrec), r = (int)(e % nrec);
  const T *u = u0 + (size_t)s * vol;
  T v = T(0);
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    int64_t idx = ridx[(size_t)r * 8 + c];
    if (idx >= 0) v += rw[(size_t)r * 8 + c] * u[idx];
  }
  traces[((size_t)s * nsteps + tl) * nrec + r] = v;
}

// Source injection and receiver sampling carried by a patch launch (nsb, ninj = 0: none).
// The sampling workgroups read p^n of this step for the step before it (trace row
// tcount[1] - tcount[2]); the injection workgroup adds this step's sources (tcount[0]).
// With advance, the last io workgroup to finish advances the step counter, as k_inject
// does.  The first-order form splits them: the gradient rows sample, the divergence rows
// inject and advance.
template <typename T>
struct PatchIo {
  const int64_t *ridx;
  const T *rw;
  int nrec, nsb;          // receivers, sampling workgroups (set by the launcher from nrs)
  int64_t nrs;            // receiver-shots to sample (0: none)
  T *traces;
  int64_t nsteps;
  const int64_t *sidx;
  const T *sw, *wavelet;
  int64_t wstride;
  int ninj;               // injection workgroups (0 or 1)
  int64_t *tcount;        // step counter (read by the io workgroups)
  int advance;            // whether the last io workgroup advances the counter
};


// sampling workgroup b of io.nsb: receiver-shots b * blockDim + tid, then every nsb
// workgroups further (the workgroups are capped, so that few of them count toward the step
// counter's advance: one atomic each)
constexpr int64_t kMaxSampleBlocks = 128;
template <typename T>
__device__ __forceinline__ void sample_block(const T *un, const PatchIo<T> &io, int b, int64_t vol) {
  const int64_t tl = io.tcount[1] - io.tcount[2];
  for (int64_t e = (int64_t)b * blockDim.x + threadIdx.x; e < io.nrs; e += (int64_t)io.nsb * blockDim.x)
    sample_receiver(un, io.ridx, io.rw, io.nrec, vol, io.traces, io.nsteps, tl, e);
}

// the end of each io workgroup (the only ones that read the step counter): the last one
// advances the counter.  Every read of the counter in the workgroup has returned (the
// barrier waits for them).  No fence: nothing written here is read by another workgroup of
// this launch (a device-scope fence would write back the L2 of each workgroup's XCD)
template <typename T>
__device__ __forceinline__ void finish_io(const PatchIo<T> &io) {
  if (!io.advance) return;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned *done = reinterpret_cast<unsigned *>(io.tcount + 3);
    if (atomicAdd(done, 1u) == (unsigned)(io.nsb + io.ninj - 1)) {
      const int64_t t = io.tcount[0];
      io.tcount[1] = t;
      io.tcount[0] = t + 1;
      *done = 0u;
    }
  }
}

}  // namespace ib
