// Launch descriptors shared by the stepping kernels and the host driver.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ib_internal.h"

namespace ib {

struct StepArgs {
  int prec;
  int ndim, M;
  int nx, ny, nz;
  int64_t pitch, vol;
  int nshots;
  int zchunk;
  const void *un;       // p^n
  void *um;             // p^{n-1} in, p^{n+1} out
  const void *K;
  const void *sx, *sy, *sz;
  // IB patch
  int64_t nib;
  const uint32_t *rec;
  const void *pinfo;          // per-point records (position, code, offset, scale)
  const int32_t *ball;
  const int32_t *delta;       // linear offsets of the ball lattice points for this layout
  const int32_t *ball_meta;   // [code][2]: start, count
  // sources / receivers
  const int64_t *sidx;
  const void *sw;
  const void *wavelet;
  int64_t wstride;
  int64_t *tcount;      // device [0] next step, [1] step being sampled, [2] first step of the call
  int nrec;
  const int64_t *ridx;
  const void *rw;
  void *traces;
  int64_t nsteps;
};

void enqueue_step(const StepArgs &a, hipStream_t st);
void enqueue_interior_only(const StepArgs &a, hipStream_t st);
void enqueue_patch_only(const StepArgs &a, hipStream_t st);
size_t pinfo_bytes(int prec);
void enqueue_make_pinfo(int prec, const int16_t *xyz, const uint32_t *roff, const void *scale, int64_t nib,
                        void *out, hipStream_t st);
void enqueue_make_delta(const int32_t *ball, int n, int64_t pitch, int64_t plane, int32_t *delta, hipStream_t st);

}  // namespace ib
