// Periodic Catmull-Rom heightfield z = H(x[, y]) (grid units) and its derivatives.
#pragma once
#include <hip/hip_runtime.h>

namespace ib {

struct SurfView {
  const double *Hs;
  int nx, ny;      // ny = 1 in 2D
  int lat;         // lateral dimensions: 1 or 2
};

__device__ __forceinline__ inline int wrapi(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

__device__ __forceinline__ void cr_weights(double t, double w[4], double dw[4], double ddw[4]) {
  double t2 = t * t, t3 = t2 * t;
  w[0] = 0.5 * (-t + 2.0 * t2 - t3);
  w[1] = 0.5 * (2.0 - 5.0 * t2 + 3.0 * t3);
  w[2] = 0.5 * (t + 4.0 * t2 - 3.0 * t3);
  w[3] = 0.5 * (-t2 + t3);
  dw[0] = 0.5 * (-1.0 + 4.0 * t - 3.0 * t2);
  dw[1] = 0.5 * (-10.0 * t + 9.0 * t2);
  dw[2] = 0.5 * (1.0 + 8.0 * t - 9.0 * t2);
  dw[3] = 0.5 * (-2.0 * t + 3.0 * t2);
  ddw[0] = 0.5 * (4.0 - 6.0 * t);
  ddw[1] = 0.5 * (-10.0 + 18.0 * t);
  ddw[2] = 0.5 * (8.0 - 18.0 * t);
  ddw[3] = 0.5 * (-2.0 + 6.0 * t);
}

// H, gradient and Hessian (xx, xy, yy) at lateral point (u, v) (v unused in 2D).
__device__ inline void surf_eval(const SurfView &s, double u, double v, double &H, double g[2], double hh[3]) {
  double ku = floor(u);
  double tu = u - ku;
  double wu[4], dwu[4], ddwu[4];
  cr_weights(tu, wu, dwu, ddwu);
  int iu = (int)ku;
  if (s.lat == 1) {
    double a = 0, b = 0, c = 0;
    for (int q = 0; q < 4; ++q) {
      double P = s.Hs[wrapi(iu - 1 + q, s.nx)];
      a += wu[q] * P;
      b += dwu[q] * P;
      c += ddwu[q] * P;
    }
    H = a;
    g[0] = b;
    g[1] = 0.0;
    hh[0] = c;
    hh[1] = 0.0;
    hh[2] = 0.0;
    return;
  }
  double kv = floor(v);
  double tv = v - kv;
  double wv[4], dwv[4], ddwv[4];
  cr_weights(tv, wv, dwv, ddwv);
  int iv = (int)kv;
  double Hv = 0, gx = 0, gy = 0, hxx = 0, hyy = 0, hxy = 0;
  for (int b = 0; b < 4; ++b) {
    const double *row = s.Hs + (size_t)wrapi(iv - 1 + b, s.ny) * s.nx;
    double r0 = 0, r1 = 0, r2 = 0;
    for (int a = 0; a < 4; ++a) {
      double P = row[wrapi(iu - 1 + a, s.nx)];
      r0 += wu[a] * P;
      r1 += dwu[a] * P;
      r2 += ddwu[a] * P;
    }
    Hv += wv[b] * r0;
    gx += wv[b] * r1;
    gy += dwv[b] * r0;
    hxx += wv[b] * r2;
    hyy += ddwv[b] * r0;
    hxy += dwv[b] * r1;
  }
  H = Hv;
  g[0] = gx;
  g[1] = gy;
  hh[0] = hxx;
  hh[1] = hxy;
  hh[2] = hyy;
}

}  // namespace ib
