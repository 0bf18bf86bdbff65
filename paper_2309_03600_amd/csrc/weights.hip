// Batched FP64 modified-stencil solves: one workgroup per immersed-boundary point.
//
// For IB point i (section "Approximating Boundary Conditions"):
//   rows of A = Taylor rows a(g - i) of the data nodes g in the ball |g - i| <= r
//               (interior and not eta-excluded), then, for every boundary point x_b
//               with |x_b - i| <= r, one row per boundary condition: the condition's
//               derivative operator applied to a, evaluated at x_b - i;
//   accept when rank(A) equals the number of basis terms, else grow r by one cell, and
//   after max_radius_steps growths drop the basis order (reading of the rank rule);
//   weights (section "Reconciliation with the Interior Numerical Discretization"):
//               y = (A^+)^T c with c = sum over exterior cross-stencil nodes e of
//               w_e a(e - i); kept for the data rows (g = 0 drops the others).
//
// GPU formulation (differs from the oracle's SVD / pseudoinverse, same mathematics):
//   A is never stored.  Its rows are generated chunk by chunk in LDS and folded into
//   the triangular factor R (A = QR) by Householder reflections of [R; chunk]; R stays
//   resident in LDS (packed upper triangle, 109.6 KB for 165 terms).  The numerical
//   rank test compares sigma_min(R) (inverse iteration) with tol * sigma_max(R) (power
//   iteration).  For full column rank (A^+)^T c = A (A^T A)^{-1} c = A R^{-1} R^{-T} c:
//   two triangular solves, then one dot product per data row with its regenerated
//   Taylor row.  This is the seminormal-equation form of the minimum-norm solution of
//   A^T y = c, which is stable when R comes from an orthogonal factorisation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "ib_internal.h"
#include "wave.h"

namespace ib {

struct SolveConst {
  int8_t exps[kMaxTerms][3];
  double w2[2 * kMaxOrder + 1];   // centred second derivative, offsets -M/2..M/2
  double ws[kMaxOrder];           // staggered first derivative, offsets -(M-1)/2..(M-1)/2
  OpSet ops[3];                   // boundary-condition rows, per unknown block
};
__constant__ SolveConst c_solve;

// A family of modified operators: which fields supply data, where the expansion point
// sits, which unknown blocks the boundary rows span, and which stencil is completed.
//   family 0: Laplacian at nodes (one field, one block);
//   family 1: staggered d/dx_g of p at the v_g node (expansion at node + e_g / 2);
//   family 2: staggered divergence of v at p nodes (one field and block per component).
struct SolveArgs {
  int family, gaxis;
  int nfields, nblocks;
  const uint8_t *fcls[3];  // node classes of each data field (bit0 interior, bit1 excluded)
  const int32_t *fball[3]; // lattice points o of the field with |o + fshift| <= r
  int fnball[3], fnwords[3], fwoff[3];
  double fshift[3][3];     // position of field node (anchor + o) relative to the expansion point, minus o
  int fblock[3];
  int baxis[3];            // family 2: axis of the velocity component of each block
  double x0off[3];         // expansion point relative to the anchor node
  const uint8_t *xcls[3];  // classes of the nodes completed by the stencil (family 1: p; 2: v_n)
  const uint8_t *cls;
  const double *bp;        // [nb][8]
  const double *bpn;       // [nb][3]
  const int64_t *col_off;  // [ncol + 1]
  const int64_t *ib_node;
  const int32_t *pending;  // IB point ids of this launch
  int npend;
  int nx, ny, nz, lat;
  int NT, Mb, M, nops;
  int nball, nwords;       // totals over the fields
  double r2;               // r^2
  double robin_scale;      // mixed surface: grid-unit coefficient = robin_scale * a(x_b) (sign: n_out vs n)
  int Rc;                  // lateral column search half-width for boundary points
  double rtol;
  int chunk;
  // per-slot scratch
  int32_t *desc;
  int desc_stride;
  double *bprel;           // [slot][maxbp][8]: relative position, normal, global index, coefficient
  int maxbp;
  // outputs indexed by position in ``pending`` (+ base)
  int out_base;
  double *wout;            // [pos][nball]
  uint32_t *mout;          // [pos][nwords]
  int32_t *status;         // [pos]: 1 accepted, 0 rank deficient, -1 overflow
  int32_t *ndata;          // [pos]
  double *sigma;           // [pos] sigma_min / sigma_max
  // optional (family 0): entries of y on the boundary-condition rows, the weights of
  // the condition values g in the modified row (null: not produced)
  // (indexed by the position in this launch, not offset by out_base)
  int32_t *fbp;            // [pos][maxbp] global index of each support boundary point
  double *fwout;           // [pos][maxbp][nops]
  int32_t *fnbp;           // [pos] support boundary points
};

__device__ __forceinline__ int wrapd(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

__device__ __forceinline__ double block_sum(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
  return t;
}

// exclusive position of this thread's flag within the block, and the block total
__device__ __forceinline__ int block_scan(int flag, int *wtot, int &total) {
  unsigned long long m = __ballot(flag);
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int pre = __popcll(m & ((1ull << lane) - 1ull));
  __syncthreads();
  if (lane == 0) wtot[wv] = __popcll(m);
  __syncthreads();
  int base = 0;
  total = 0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
    if (i < wv) base += wtot[i];
    total += wtot[i];
  }
  return base + pre;
}

__device__ __forceinline__ int ridx(int i, int j, int NT) {  // packed upper triangle, row-major
  return i * NT - (i * (i - 1)) / 2 + (j - i);
}

template <int CH>
__launch_bounds__(768)   // a lane quad per column, at most 192 columns
__global__ void k_solve(SolveArgs a) {
  extern __shared__ double smem[];
  const int NTB = a.NT;                 // basis terms per block
  const int NT = a.NT * a.nblocks;      // unknowns (columns of A)
  constexpr int nb = CH;
  const int tid = threadIdx.x;
  const int nth = blockDim.x;
  const int D1 = a.Mb + 1;
  double *R = smem;                                   // NT(NT+1)/2, packed upper triangle
  double *pw = R + NT * (NT + 1) / 2;                 // CH x 3 x D1 power tables of the chunk rows
  double *nrm = pw + nb * 3 * D1;                     // CH x 3 normals of the chunk rows
  double *vcol = nrm + nb * 3;                        // 2 x CH reflector columns (double buffered)
  double *vsc = vcol + 2 * nb;                        // 2 x 2 reflector scalars
  double *C = vsc + 4;                                // NT: the published solution z
  double *red = C + 2 * NT;                           // 16 (C holds z, then 1 / R_kk)
  int *iscr = (int *)(red + 16);                      // 16 ints
  __shared__ int rowop[64];
  __shared__ int rowbp[64];
  __shared__ double rowrob[64];   // mixed-surface coefficient of each chunk row

  const int pos = blockIdx.x;
  const int slot = blockIdx.x;
  if (pos >= a.npend) return;
  const int out = a.out_base + pos;
  const int64_t node = a.ib_node[a.pending[pos]];
  const int x0 = (int)(node % a.nx);
  const int64_t rr = node / a.nx;
  const int y0 = (int)(rr % a.ny);
  const int z0 = (int)(rr / a.ny);
  int32_t *desc = a.desc + (size_t)slot * a.desc_stride;
  double *bpr = a.bprel + (size_t)slot * a.maxbp * 8;
  uint32_t *mask = a.mout + (size_t)out * a.nwords;

  // ---- data rows: lattice points of each field that are interior and not excluded ----
  int ndata = 0;
  for (int f = 0; f < a.nfields; ++f) {
    const int32_t *fb = a.fball[f];
    const uint8_t *fc = a.fcls[f];
    uint32_t *fmask = mask + a.fwoff[f];
    for (int b0 = 0; b0 < a.fnball[f]; b0 += nth) {
      int b = b0 + tid;
      int flag = 0;
      if (b < a.fnball[f]) {
        uint32_t v = (uint32_t)fb[b];
        int dx = (int8_t)(v & 255), dy = (int8_t)((v >> 8) & 255), dz = (int8_t)((v >> 16) & 255);
        int zz = z0 + dz;
        if (zz >= 0 && zz < a.nz) {
          int64_t g = ((int64_t)zz * a.ny + wrapd(y0 + dy, a.ny)) * a.nx + wrapd(x0 + dx, a.nx);
          uint8_t c = fc[g];
          flag = ((c & 1) && !(c & 2)) ? 1 : 0;
        }
      }
      int total;
      int p = block_scan(flag, iscr, total);
      if (flag && ndata + p < a.desc_stride) desc[ndata + p] = (f << 16) | b;
      unsigned long long bal = __ballot(flag);
      int lane = tid & 63;
      if (lane == 0 && b < a.fnball[f]) fmask[b >> 5] = (uint32_t)(bal & 0xffffffffull);
      if (lane == 32 && b < a.fnball[f]) fmask[b >> 5] = (uint32_t)(bal >> 32);
      ndata += total;
    }
  }
  const double xc0 = x0 + a.x0off[0], yc0 = y0 + a.x0off[1], zc0 = z0 + a.x0off[2];
  // ---- boundary points within the radius --------------------------------------------
  int nbp = 0;
  const int side = 2 * a.Rc + 1;
  const int ncols = (a.lat == 2) ? side * side : side;
  for (int c0 = 0; c0 < ncols; c0 += nth) {
    int cidx = c0 + tid;
    int cnt = 0;
    int64_t j0 = 0, j1 = 0;
    if (cidx < ncols) {
      int dx = cidx % side - a.Rc;
      int dy = (a.lat == 2) ? cidx / side - a.Rc : 0;
      int64_t col = (int64_t)wrapd(y0 + dy, a.ny) * a.nx + wrapd(x0 + dx, a.nx);
      j0 = a.col_off[col];
      j1 = a.col_off[col + 1];
      for (int64_t j = j0; j < j1; ++j) {
        const double *p = a.bp + j * 8 + 3;
        double rx = p[0] - xc0, ry = p[1] - yc0, rz = p[2] - zc0;
        rx -= a.nx * rint(rx / a.nx);
        if (a.lat == 2) ry -= a.ny * rint(ry / a.ny);
        if (rx * rx + ry * ry + rz * rz <= a.r2) ++cnt;
      }
    }
    // exclusive scan of counts (small: serial over waves via LDS)
    __syncthreads();
    __shared__ int cnts[1024];
    cnts[tid] = cnt;
    __syncthreads();
    if (tid == 0) {
      int s = 0;
      for (int i = 0; i < nth; ++i) {
        int t = cnts[i];
        cnts[i] = s;
        s += t;
      }
      iscr[8] = s;
    }
    __syncthreads();
    int w = nbp + cnts[tid];
    int tot = iscr[8];
    if (cnt > 0) {
      for (int64_t j = j0; j < j1; ++j) {
        const double *p = a.bp + j * 8 + 3;
        double rx = p[0] - xc0, ry = p[1] - yc0, rz = p[2] - zc0;
        rx -= a.nx * rint(rx / a.nx);
        if (a.lat == 2) ry -= a.ny * rint(ry / a.ny);
        if (rx * rx + ry * ry + rz * rz <= a.r2) {
          if (w < a.maxbp) {
            double *q = bpr + (size_t)w * 8;
            q[0] = rx;
            q[1] = ry;
            q[2] = rz;
            q[3] = a.bpn[j * 3 + 0];
            q[4] = a.bpn[j * 3 + 1];
            q[5] = a.bpn[j * 3 + 2];
            q[6] = (double)j;
            q[7] = a.robin_scale * a.bp[j * 8 + 6];
          }
          ++w;
        }
      }
    }
    nbp += tot;
    __syncthreads();
  }
  if (nbp > a.maxbp || ndata > a.desc_stride || NT > 192) {
    if (tid == 0) {
      a.status[out] = -1;
      a.ndata[out] = ndata;
    }
    return;
  }
  const int m = ndata + nbp * a.nops;
  if (m < NT) {   // fewer rows than unknowns: rank deficient
    if (tid == 0) {
      a.status[out] = 0;
      a.ndata[out] = ndata;
      a.sigma[out] = 0.0;
    }
    return;
  }
  __threadfence_block();
  __syncthreads();

  // ---- streamed Householder QR of A into R ------------------------------------------
  // Four threads (a lane quad) own column j of the current row chunk, every fourth row
  // each (interleaved, so that the quad's LDS reads of rows and reflectors hit adjacent
  // words), in registers.  Column step k: the quad of column k forms the reflector of
  // [R_kk; chunk column k] (quad sums by DPP, identical in its four lanes) and publishes it
  // in LDS (double buffered); every quad j > k applies it to [R_kj; its column].  Quarter
  // rows keep the per-thread dependency chains short, and the larger workgroup hides
  // latency with more wavefronts on the CU that R's LDS footprint limits to one point.
  constexpr int RQ = CH / 4;                      // chunk rows per quarter
  const int cjx = tid >> 2, qd = tid & 3;         // column and quarter of this thread
  for (int i = tid; i < NT * (NT + 1) / 2; i += nth) R[i] = 0.0;
  const int bj = (cjx < NT) ? cjx / NTB : 0;      // unknown block of column cjx
  const int tj = (cjx < NT) ? cjx - bj * NTB : 0; // basis term of column cjx
  const int8_t ej0 = c_solve.exps[tj][0];
  const int8_t ej1 = c_solve.exps[tj][1];
  const int8_t ej2 = c_solve.exps[tj][2];
  auto quad_sum = [](double v) {
    v += dpp_mov<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_mov<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    return v;
  };
  __syncthreads();
  for (int r0 = 0; r0 < m; r0 += nb) {
    const int nr = min(nb, m - r0);
    // row kinds and per-row power tables  delta_n^k / k!
    if (tid < nr) {
      int r = r0 + tid;
      double d[3];
      if (r < ndata) {
        const int f = desc[r] >> 16;
        uint32_t v = (uint32_t)a.fball[f][desc[r] & 0xffff];
        d[0] = (int8_t)(v & 255) + a.fshift[f][0];
        d[1] = (int8_t)((v >> 8) & 255) + a.fshift[f][1];
        d[2] = (int8_t)((v >> 16) & 255) + a.fshift[f][2];
        rowop[tid] = -1 - a.fblock[f];
        rowrob[tid] = 0.0;
        nrm[tid * 3 + 0] = nrm[tid * 3 + 1] = nrm[tid * 3 + 2] = 0.0;
      } else {
        int rb = r - ndata;
        int bi = rb / a.nops;
        rowop[tid] = rb % a.nops;
        rowbp[tid] = bi;
        const double *q = bpr + (size_t)bi * 8;
        rowrob[tid] = q[7];
        d[0] = q[0];
        d[1] = q[1];
        d[2] = q[2];
        nrm[tid * 3 + 0] = q[3];
        nrm[tid * 3 + 1] = q[4];
        nrm[tid * 3 + 2] = q[5];
      }
      for (int n = 0; n < 3; ++n) {
        double *t = pw + (tid * 3 + n) * D1;
        t[0] = 1.0;
        for (int k = 1; k < D1; ++k) t[k] = t[k - 1] * d[n] / (double)k;
      }
    }
    __syncthreads();
    double cj[RQ];
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
      const int i = 4 * r + qd;
      double v = 0.0;
      if (i < nr && cjx < NT) {
        const double *p = pw + i * 3 * D1;
        const int op = rowop[i];
        if (op < 0) {
          v = (-1 - op == bj) ? p[ej0] * p[D1 + ej1] * p[2 * D1 + ej2] : 0.0;
        } else {
          const OpSet &OS = c_solve.ops[bj];
          const int nt_ = OS.nterms[op];
          for (int q = 0; q < nt_; ++q) {
            const OpTerm &T = OS.term[op][q];
            const int a0 = ej0 - T.beta[0], a1 = ej1 - T.beta[1], a2 = ej2 - T.beta[2];
            if (a0 < 0 || a1 < 0 || a2 < 0) continue;
            double cf = T.coef;
            if (T.normal_axis >= 0) cf *= nrm[i * 3 + T.normal_axis];
            if (T.scaled) cf *= rowrob[i];
            v += cf * p[a0] * p[D1 + a1] * p[2 * D1 + a2];
          }
        }
      }
      cj[r] = v;
    }
    for (int k = 0; k < NT; ++k) {
      double *vc = vcol + (k & 1) * nb;
      double *sc = vsc + (k & 1) * 2;
      if (cjx == k) {
        double part = 0.0;
#pragma unroll
        for (int r = 0; r < RQ; ++r) part += cj[r] * cj[r];
        const double nsq = quad_sum(part);
        const double rkk = R[ridx(k, k, NT)];
        double al, v0;
        // a chunk column of norm below 1e-150 is taken as zero: its reflector would move R by
        // less than the rounding of its other entries, and al * v0 below must stay a normal
        // number (its underflow to zero made f infinite and R non-finite)
        if (!(nsq > 1e-300)) {
          al = rkk;
          v0 = 0.0;
        } else {
          const double nn = sqrt(rkk * rkk + nsq);
          al = (rkk >= 0.0) ? -nn : nn;
          v0 = rkk - al;
        }
        if (qd == 0) {
          sc[0] = al;
          sc[1] = v0;
          R[ridx(k, k, NT)] = al;
        }
#pragma unroll
        for (int r = 0; r < RQ; ++r) vc[4 * r + qd] = cj[r];
      }
      __syncthreads();
      const double al = sc[0], v0 = sc[1];
      if (cjx > k && cjx < NT && v0 != 0.0) {
        const int rk = ridx(k, cjx, NT);
        const double rkj = R[rk];
        double part = (qd == 0) ? v0 * rkj : 0.0;
#pragma unroll
        for (int r = 0; r < RQ; ++r) part += vc[4 * r + qd] * cj[r];
        const double f = quad_sum(part) / (al * v0);
        if (qd == 0) R[rk] = rkj + f * v0;
#pragma unroll
        for (int r = 0; r < RQ; ++r) cj[r] += f * vc[4 * r + qd];
      }
    }
    __syncthreads();
  }

  // ---- numerical rank and the solve --------------------------------------------------
  // Vectors of length NT <= 192 live in registers (entry j in lane j % 64, slot j / 64);
  // triangular solves and mat-vecs broadcast one entry per step with readlane, so a
  // wavefront needs no workgroup barrier inside them.  sigma_max (power iteration) runs on
  // wavefront 1 while wavefront 0 runs the inverse iteration for sigma_min; wavefront 0
  // then decides and solves.  The diagonal's reciprocals are formed once.
  double *zv = C;            // reuse the chunk buffer for the published solution
  double *dinv = C + NT;     // 1 / R_kk
  for (int k = tid; k < NT; k += nth) dinv[k] = 1.0 / R[ridx(k, k, NT)];
  __syncthreads();
  const int wvi = tid >> 6, lane = tid & 63;
  const bool two = nth >= 128;
  auto bcast = [](double v, int src) {
    int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
  };
  auto get = [&](const double x[3], int k) { return bcast(k < 64 ? x[0] : (k < 128 ? x[1] : x[2]), k & 63); };
  auto wsum = [](double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
  };
  // R^T w = x in place (x becomes w)
  auto solve_rt = [&](double x[3]) {
    for (int k = 0; k < NT; ++k) {
      const double wk = get(x, k) * dinv[k];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int j = lane + 64 * q;
        if (j > k && j < NT) x[q] -= R[ridx(k, j, NT)] * wk;
        if (j == k) x[q] = wk;
      }
    }
  };
  // R z = w in place
  auto solve_r = [&](double x[3]) {
    for (int k = NT - 1; k >= 0; --k) {
      const double zk = get(x, k) * dinv[k];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int j = lane + 64 * q;
        if (j < k) x[q] -= R[ridx(j, k, NT)] * zk;
        if (j == k) x[q] = zk;
      }
    }
  };
  const double inv_sqrt = 1.0 / sqrt((double)NT);
  // sigma_max: power iteration on R^T R
  auto power = [&]() {
    double x[3], y[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) x[q] = (lane + 64 * q < NT) ? inv_sqrt : 0.0;
    double smax2 = 0.0;
    for (int it = 0; it < 8; ++it) {
#pragma unroll
      for (int q = 0; q < 3; ++q) y[q] = 0.0;
      for (int j = 0; j < NT; ++j) {      // y = R x
        const double xj = get(x, j);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const int i = lane + 64 * q;
          if (i <= j && i < NT) y[q] += R[ridx(i, j, NT)] * xj;
        }
      }
      double x2[3] = {0.0, 0.0, 0.0};
      for (int i = 0; i < NT; ++i) {      // x2 = R^T y
        const double yi = get(y, i);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const int j = lane + 64 * q;
          if (j >= i && j < NT) x2[q] += R[ridx(i, j, NT)] * yi;
        }
      }
      const double nn = sqrt(wsum(x2[0] * x2[0] + x2[1] * x2[1] + x2[2] * x2[2]));
      smax2 = nn;
#pragma unroll
      for (int q = 0; q < 3; ++q) x[q] = (nn > 0.0) ? x2[q] / nn : 0.0;
    }
    return smax2;
  };
  if (wvi == (two ? 1 : 0)) {
    const double s2 = power();
    if (lane == 0) red[0] = s2;
  }
  double x[3];
  double smin2 = 0.0;
  if (wvi == 0) {
    // sigma_min: inverse iteration on R^T R from an alternating start
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int j = lane + 64 * q;
      x[q] = (j < NT) ? ((j & 1) ? -inv_sqrt : inv_sqrt) : 0.0;
    }
    for (int it = 0; it < 6; ++it) {
      solve_rt(x);
      solve_r(x);
      const double nn = sqrt(wsum(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]));
      if (!isfinite(nn) || !(nn > 0.0)) {
        smin2 = 0.0;
        break;
      }
      smin2 = 1.0 / nn;
#pragma unroll
      for (int q = 0; q < 3; ++q) x[q] /= nn;
    }
  }
  __syncthreads();
  if (wvi == 0) {
    const double smax = sqrt(red[0]), smin = sqrt(smin2);
    const double tol = (a.rtol > 0.0) ? a.rtol : (double)max(m, NT) * 2.220446049250313e-16;
    const bool full = (smin > tol * smax) && isfinite(smin) && isfinite(smax) && smax > 0.0;
    if (lane == 0) {
      a.status[out] = full ? 1 : 0;
      a.ndata[out] = ndata;
      a.sigma[out] = (smax > 0.0) ? smin / smax : 0.0;
      iscr[9] = full ? 1 : 0;
    }
    if (full) {
      // c = sum of w_e a(x_e - x_0) over the exterior nodes the completed stencil reads
      // (family 0: Laplacian cross; 1: staggered gradient; 2: staggered divergence,
      // one block per velocity component), then R^T w = c, R z = w
      const int half = a.M / 2;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int col = lane + 64 * q;
        double cv = 0.0;
        if (col < NT) {
          const int blk = col / NTB, t = col - blk * NTB;
          const int8_t *ex = c_solve.exps[t];
          auto pure_in = [&](int n) {
            for (int qq = 0; qq < 3; ++qq)
              if (qq != n && ex[qq] != 0) return false;
            return true;
          };
          auto mono = [&](int n, double rel) {
            double v = 1.0;
            for (int pp = 1; pp <= ex[n]; ++pp) v = v * rel / (double)pp;
            return v;
          };
          auto exterior = [&](const uint8_t *cl, int xx, int yy, int zz) {
            if (zz < 0 || zz >= a.nz) return false;
            return !(cl[((int64_t)zz * a.ny + wrapd(yy, a.ny)) * a.nx + wrapd(xx, a.nx)] & 1);
          };
          if (a.family == 0) {
            for (int n = 0; n < 3; ++n) {
              if (a.lat == 1 && n == 1) continue;
              if (!pure_in(n)) continue;
              for (int k = -half; k <= half; ++k) {
                if (k == 0) continue;
                const int xx = x0 + (n == 0 ? k : 0), yy = y0 + (n == 1 ? k : 0), zz = z0 + (n == 2 ? k : 0);
                if (!exterior(a.cls, xx, yy, zz)) continue;
                cv += c_solve.w2[k + half] * mono(n, (double)k);
              }
            }
          } else if (a.family == 1) {
            const int n = a.gaxis;
            if (pure_in(n)) {
              for (int k = -half + 1; k <= half; ++k) {
                const int xx = x0 + (n == 0 ? k : 0), yy = y0 + (n == 1 ? k : 0), zz = z0 + (n == 2 ? k : 0);
                if (!exterior(a.xcls[0], xx, yy, zz)) continue;
                cv += c_solve.ws[k + half - 1] * mono(n, (double)k - 0.5);
              }
            }
          } else {
            const int n = a.baxis[blk];
            if (pure_in(n)) {
              for (int k = -half; k <= half - 1; ++k) {
                const int xx = x0 + (n == 0 ? k : 0), yy = y0 + (n == 1 ? k : 0), zz = z0 + (n == 2 ? k : 0);
                if (!exterior(a.xcls[blk], xx, yy, zz)) continue;
                cv += c_solve.ws[k + half] * mono(n, (double)k + 0.5);
              }
            }
          }
        }
        x[q] = cv;
      }
      solve_rt(x);
      solve_r(x);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int t = lane + 64 * q;
        if (t < NT) zv[t] = x[q];
      }
    }
  }
  __syncthreads();
  if (!iscr[9]) return;
  double *yv = zv;
  // y_j = a_j . z for the data rows
  double *wo = a.wout + (size_t)out * a.nball;
  for (int j = tid; j < ndata; j += nth) {
    const int f = desc[j] >> 16;
    uint32_t v = (uint32_t)a.fball[f][desc[j] & 0xffff];
    double d[3] = {(double)(int8_t)(v & 255) + a.fshift[f][0], (double)(int8_t)((v >> 8) & 255) + a.fshift[f][1],
                   (double)(int8_t)((v >> 16) & 255) + a.fshift[f][2]};
    const double *zb = yv + a.fblock[f] * NTB;
    double p[3][kMaxOrder + 1];
    for (int n = 0; n < 3; ++n) {
      p[n][0] = 1.0;
      for (int k = 1; k < D1; ++k) p[n][k] = p[n][k - 1] * d[n] / (double)k;
    }
    double s = 0.0;
    for (int t = 0; t < NTB; ++t) {
      const int8_t *ex = c_solve.exps[t];
      s += p[0][ex[0]] * p[1][ex[1]] * p[2][ex[2]] * zb[t];
    }
    wo[j] = s;
  }
  // y on the boundary-condition rows: row (b, op) . z with the row regenerated exactly as
  // in the factorisation (one block: the second-order form's Laplacian family)
  if (a.fwout && a.nblocks == 1) {
    int32_t *fb = a.fbp + (size_t)pos * a.maxbp;
    double *fw = a.fwout + (size_t)pos * a.maxbp * a.nops;
    if (tid == 0) a.fnbp[pos] = nbp;
    const OpSet &OS = c_solve.ops[0];
    for (int r = tid; r < nbp * a.nops; r += nth) {
      const int bi = r / a.nops, op = r - bi * a.nops;
      const double *q = bpr + (size_t)bi * 8;
      if (op == 0) fb[bi] = (int32_t)q[6];
      double p[3][kMaxOrder + 1];
      for (int n = 0; n < 3; ++n) {
        p[n][0] = 1.0;
        for (int k = 1; k < D1; ++k) p[n][k] = p[n][k - 1] * q[n] / (double)k;
      }
      double s = 0.0;
      for (int t = 0; t < NTB; ++t) {
        const int8_t *ex = c_solve.exps[t];
        double v = 0.0;
        for (int u = 0; u < OS.nterms[op]; ++u) {
          const OpTerm &T = OS.term[op][u];
          const int a0 = ex[0] - T.beta[0], a1 = ex[1] - T.beta[1], a2 = ex[2] - T.beta[2];
          if (a0 < 0 || a1 < 0 || a2 < 0) continue;
          double cf = T.coef;
          if (T.normal_axis >= 0) cf *= q[3 + T.normal_axis];
          if (T.scaled) cf *= q[7];
          v += cf * p[0][a0] * p[1][a1] * p[2][a2];
        }
        s += v * yv[t];
      }
      fw[r] = s;
    }
  }
}

// Gather accepted points of one round into the final tables.
__global__ void k_pack(int nacc, const int32_t *acc_pos, const int32_t *acc_id, const double *wout, int nball,
                       const uint32_t *mout, int nwords, const int32_t *woff, const int32_t *nw,
                       const uint32_t *roff32, const uint32_t *roff64, double *w64, uint32_t *rec32,
                       uint32_t *rec64) {
  int a = blockIdx.x;
  if (a >= nacc) return;
  int pos = acc_pos[a], id = acc_id[a];
  const double *src = wout + (size_t)pos * nball;
  const uint32_t *msk = mout + (size_t)pos * nwords;
  int n = nw[id];
  uint32_t o32 = roff32[id], o64 = roff64[id];
  int nw64 = (nwords + 1) & ~1;
  for (int t = threadIdx.x; t < nwords; t += blockDim.x) rec32[o32 + t] = msk[t];
  for (int t = threadIdx.x; t < nw64; t += blockDim.x) rec64[o64 + t] = (t < nwords) ? msk[t] : 0u;
  float *f32 = reinterpret_cast<float *>(rec32 + o32 + nwords);
  double *f64 = reinterpret_cast<double *>(rec64 + o64 + nw64);
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    double v = src[t];
    w64[woff[id] + t] = v;
    f32[t] = (float)v;
    f64[t] = v;
  }
}

// Condition-value weights of the accepted points of one launch, compacted: entry e of
// point a is (boundary point << 3 | condition) and its weight.
__global__ void k_pack_bc(int nacc, const int32_t *apos, const int64_t *aoff, const int32_t *fbp, const double *fw,
                          const int32_t *fnbp, int maxbp, int nops, int32_t *oidx, double *ow) {
  const int a = blockIdx.x;
  if (a >= nacc) return;
  const int pos = apos[a];
  const int n = fnbp[pos] * nops;
  const int64_t o = aoff[a];
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int bi = e / nops, q = e - bi * nops;
    oidx[o + e] = (fbp[(size_t)pos * maxbp + bi] << 3) | q;
    ow[o + e] = fw[(size_t)pos * maxbp * nops + e];
  }
}

// Dense-range records: per point, the weights of every support-ball lattice point from
// the first to the last data point (zero where the lattice point is not data), so a
// kernel can stream them without decoding the mask.
__global__ void k_mask_range(int64_t nib, const uint32_t *rec32, const uint32_t *roff32, const int16_t *xyz,
                             const int32_t *ball_meta, int32_t *first, int32_t *count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nib) return;
  const int code = xyz[i * 4 + 3];
  const int nb = ball_meta[2 * code + 1];
  const uint32_t *m = rec32 + roff32[i];
  int f = -1, l = -1;
  for (int b = 0; b < nb; ++b) {
    if ((m[b >> 5] >> (b & 31)) & 1u) {
      if (f < 0) f = b;
      l = b;
    }
  }
  first[i] = (f < 0) ? 0 : f;
  count[i] = (f < 0) ? 0 : l - f + 1;
}

__global__ void k_dense(int64_t nib, const uint32_t *rec32, const uint32_t *roff32, const int32_t *meta,
                        const double *w64, const int32_t *first, const int32_t *count, const uint32_t *doff,
                        float *d32, double *d64) {
  const int64_t i = blockIdx.x;
  if (i >= nib) return;
  const int lane = threadIdx.x;     // one wavefront per point
  const uint32_t *m = rec32 + roff32[i];
  const int f = first[i], n = count[i];
  const int64_t woff = meta[i * 4 + 3];
  // data points before the range start
  int base = 0;
  for (int b = lane; b < f; b += 64) base += (int)((m[b >> 5] >> (b & 31)) & 1u);
  for (int o = 32; o > 0; o >>= 1) base += __shfl_xor(base, o);
  for (int e0 = 0; e0 < n; e0 += 64) {
    const int e = e0 + lane;
    const int b = f + e;
    const int bit = (e < n) ? (int)((m[b >> 5] >> (b & 31)) & 1u) : 0;
    const unsigned long long bal = __ballot(bit);
    const int k = base + __popcll(bal & ((1ull << lane) - 1ull));
    if (e < n) {
      const double v = bit ? w64[woff + k] : 0.0;
      d32[doff[i] + e] = (float)v;
      d64[doff[i] + e] = v;
    }
    base += __popcll(bal);
  }
}

// ---- column-run records (3D supports of radius 4 and 4.5, the LDS-tiled patch) --------
// A support ball is a set of depth columns (dx, dy), each spanning dz in [-zr, zr].  The
// data nodes of a column (interior and not excluded) lie at or below the first data node
// of their grid column, zfirst(x + dx, y + dy): the column contributes the run
// [a, zr], a = max(zfirst - z, -zr), and a node of the run that is not data (a rare node
// excluded below the first data node, or a node below the box) gets a zero weight.  Column
// c belongs to lane c of a wavefront; the radius-4.5 ball has 69 columns, and its five
// extra single-node columns (zr = 0) go to lanes 0..4, whose own columns are short.  The
// record holds each lane's run (then its extra node) contiguously, lanes in order, so a
// lane's entries start at the count of its lower lanes' entries (a ballot prefix count) and
// are read with a few wide loads; no per-weight offsets are stored.

// first data plane of every grid column (nz where a column has none)
__global__ void k_zfirst(const uint8_t *cls, int nx, int ny, int nz, int16_t *zf) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (int64_t)nx * ny) return;
  int z = 0;
  for (; z < nz; ++z) {
    const uint8_t v = cls[(int64_t)z * nx * ny + c];
    if ((v & 1) && !(v & 2)) break;
  }
  zf[c] = (int16_t)z;
}

// the run of the lane's column (and of its extra column) for IB point i; len = -1: no column
struct ColRun {
  int dx, dy, a, len;
};
__device__ __forceinline__ ColRun col_run(int32_t col, const int16_t *zf, int x, int y, int z, int nx, int ny) {
  ColRun r{0, 0, 0, 0};
  if (col == kNoColumn) return r;
  r.dx = (int8_t)(col & 255);
  r.dy = (int8_t)((col >> 8) & 255);
  const int zr = (col >> 16) & 255;
  int xx = x + r.dx, yy = y + r.dy;
  xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
  yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
  r.a = max((int)zf[(int64_t)yy * nx + xx] - z, -zr);
  r.len = max(0, zr - r.a + 1);
  return r;
}

// the lane's main column and extra column for a support of radius code 8 or 9
__device__ __forceinline__ void lane_columns(const int32_t *coltab, int code, int lane, int32_t &mc, int32_t &ec) {
  mc = (code == 9) ? coltab[lane] : (lane < kColumns8 ? coltab[kColumns9 + lane] : kNoColumn);
  ec = (code == 9 && lane < kColumns9 - 64) ? coltab[64 + lane] : kNoColumn;
}

// entries per IB point (-1 for supports the tiled patch does not take)
__global__ void k_col_count(int64_t nib, const int16_t *xyz, const int16_t *zf, const int32_t *coltab, int nx, int ny,
                            int32_t *cnt) {
  const int64_t i = blockIdx.x;
  if (i >= nib) return;
  const int lane = threadIdx.x;
  const int code = xyz[i * 4 + 3];
  if (code != 8 && code != 9) {
    if (lane == 0) cnt[i] = -1;
    return;
  }
  const int x = xyz[i * 4], y = xyz[i * 4 + 1], z = xyz[i * 4 + 2];
  int32_t mc, ec;
  lane_columns(coltab, code, lane, mc, ec);
  int n = col_run(mc, zf, x, y, z, nx, ny).len + col_run(ec, zf, x, y, z, nx, ny).len;
  for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o);
  if (lane == 0) cnt[i] = n;
}

// entries of one IB point: weights from the compact record (data-membership mask + the
// data nodes' weights in ball order), zero at non-data nodes of the runs; err counts the
// points whose data nodes are not all covered by the runs (none, by the construction)
__global__ void k_col_pack(int64_t nib, const int16_t *xyz, const int32_t *meta, const uint32_t *rec32,
                           const uint32_t *roff32, const double *w64, const int16_t *zf, const int32_t *coltab,
                           const int16_t *inv, const int32_t *ball_meta, int nx, int ny, int nz, const uint32_t *off,
                           const int32_t *cnt, float *c32, double *c64, int32_t *err) {
  const int64_t i = blockIdx.x;
  if (i >= nib || cnt[i] < 0) return;
  const int lane = threadIdx.x;
  const int code = xyz[i * 4 + 3];
  const int x = xyz[i * 4], y = xyz[i * 4 + 1], z = xyz[i * 4 + 2];
  const int16_t *iv = inv + (code == 9 ? 0 : 729);
  const int nb = ball_meta[2 * code + 1];
  const uint32_t *m = rec32 + roff32[i];
  const double *wv = w64 + meta[i * 4 + 3];
  const int nw = meta[i * 4 + 2];
  int32_t mc, ec;
  lane_columns(coltab, code, lane, mc, ec);
  const ColRun R = col_run(mc, zf, x, y, z, nx, ny);
  const ColRun E = col_run(ec, zf, x, y, z, nx, ny);
  // the weight of the node (dx, dy, dz) of this point's ball: 0 unless it is a data node
  auto weight = [&](int dx, int dy, int dz, int &covered) -> double {
    if (z + dz >= nz) return 0.0;
    const int b = iv[((dz + 4) * 9 + (dy + 4)) * 9 + (dx + 4)];
    if (b < 0 || b >= nb || !((m[b >> 5] >> (b & 31)) & 1u)) return 0.0;
    int rank = 0;
    for (int q = 0; q < (b >> 5); ++q) rank += __popc(m[q]);
    rank += __popc(m[b >> 5] & ((1u << (b & 31)) - 1u));
    ++covered;
    return wv[rank];
  };
  // this lane's first entry: the entries of the lower lanes (one ballot per entry count)
  const int len = R.len + E.len;
  int pos = 0, tot = 0;
  for (int k = 0; k < 2 * 4 + 2; ++k) {
    const unsigned long long bal = __ballot(len > k);
    pos += __popcll(bal & ((1ull << lane) - 1ull));
    tot += __popcll(bal);
  }
  int covered = 0;
  const uint32_t o = off[i] + (uint32_t)pos;
  for (int k = 0; k < len; ++k) {
    const double v = (k < R.len) ? weight(R.dx, R.dy, R.a + k, covered) : weight(E.dx, E.dy, 0, covered);
    c32[o + k] = (float)v;
    c64[o + k] = v;
  }
  for (int s = 32; s > 0; s >>= 1) covered += __shfl_xor(covered, s);
  if (lane == 0 && (covered != nw || tot != cnt[i])) atomicAdd(err, 1);
}

// threads of a k_solve workgroup: a lane quad per column of A, whole wavefronts
static int solve_threads(int ncols) { return std::min(768, std::max(64, (4 * ncols + 63) / 64 * 64)); }

struct RoundResult {
  int code, k, Mb;
  std::vector<int32_t> acc_pos, acc_id;
  double *wout = nullptr;
  uint32_t *mout = nullptr;
  int nball = 0, nwords = 0;
};

// Ball lattice tables (all radius codes up to max_code + 2) on the device.
ib_status upload_ball_tables(ib_weights *w, hipStream_t st) {
  w->balls.build(w->ndim, w->max_code + 2);
  ib_status s;
  if ((s = dalloc_t(&w->ball, w->balls.packed.size()))) return s;
  IB_HIP(hipMemcpyAsync(w->ball, w->balls.packed.data(), w->balls.packed.size() * 4, hipMemcpyHostToDevice, st));
  std::vector<int32_t> bm(2 * (kMaxRadiusCode + 2), 0);
  for (int c = 0; c <= kMaxRadiusCode + 1; ++c) {
    bm[2 * c] = w->balls.start[c];
    bm[2 * c + 1] = w->balls.count[c];
  }
  if ((s = dalloc_t(&w->ball_meta, bm.size()))) return s;
  IB_HIP(hipMemcpy(w->ball_meta, bm.data(), bm.size() * 4, hipMemcpyHostToDevice));
  return IB_OK;
}

// Dense-range records (weights of every ball lattice point from the first to the last data
// point of each support) from the compact records.
ib_status build_dense_records(ib_weights *w, hipStream_t st) {
  const int64_t nib = w->nib;
  ib_status s;
  {
    int32_t *d_first = nullptr, *d_count = nullptr;
    uint32_t *d_doff = nullptr;
    if ((s = dalloc_t(&d_first, std::max<int64_t>(nib, 1))) || (s = dalloc_t(&d_count, std::max<int64_t>(nib, 1))) ||
        (s = dalloc_t(&d_doff, std::max<int64_t>(nib, 1))))
      return s;
    if (nib)
      hipLaunchKernelGGL(k_mask_range, dim3((unsigned)((nib + 255) / 256)), dim3(256), 0, st, nib, w->rec32,
                         w->rec_off32, w->ib_xyz, w->ball_meta, d_first, d_count);
    std::vector<int32_t> hf(nib), hc(nib);
    std::vector<uint32_t> ho(nib);
    IB_HIP(hipMemcpyAsync(hf.data(), d_first, nib * 4, hipMemcpyDeviceToHost, st));
    IB_HIP(hipMemcpyAsync(hc.data(), d_count, nib * 4, hipMemcpyDeviceToHost, st));
    IB_HIP(hipStreamSynchronize(st));
    // each record starts at an even offset (a zero pads odd lengths), so that the tiled
    // patch can load FP32 weights in pairs
    int64_t sd = 0;
    for (int64_t i = 0; i < nib; ++i) {
      ho[i] = (uint32_t)sd;
      sd += (hc[i] + 1) & ~1;
    }
    if (sd >= (int64_t)UINT32_MAX) {
      set_error("dense stencil table too large");
      return IB_ERR_ARG;
    }
    w->dense_words = sd;
    w->stats.dense_weights = sd;
    if ((s = dalloc_t(&w->dense32, std::max<int64_t>(sd, 2))) || (s = dalloc_t(&w->dense64, std::max<int64_t>(sd, 2))))
      return s;
    IB_HIP(hipMemsetAsync(w->dense32, 0, std::max<int64_t>(sd, 2) * sizeof(float), st));
    IB_HIP(hipMemsetAsync(w->dense64, 0, std::max<int64_t>(sd, 2) * sizeof(double), st));
    IB_HIP(hipMemcpyAsync(d_doff, ho.data(), nib * 4, hipMemcpyHostToDevice, st));
    if (nib)
      hipLaunchKernelGGL(k_dense, dim3((unsigned)nib), dim3(64), 0, st, nib, w->rec32, w->rec_off32, w->ib_meta,
                         w->w64, d_first, d_count, d_doff, w->dense32, w->dense64);
    IB_HIP(hipGetLastError());
    IB_HIP(hipStreamSynchronize(st));
    w->dense_first = d_first;
    w->dense_count = d_count;
    w->dense_off = d_doff;
  }
  return IB_OK;
}

// Column-run records of the 3D supports of radius 4 and 4.5 (see k_col_pack).
ib_status build_column_records(ib_weights *w, hipStream_t st) {
  if (w->ndim != 3 || w->nib == 0) return IB_OK;
  const int64_t nib = w->nib, ncols = w->nx * w->ny;
  if (w->nz > 32767) {
    set_error("column-run records need nz < 32768");
    return IB_ERR_ARG;
  }
  // column tables: code 9 (69 columns, the five extra single-node ones last), then code 8
  std::vector<int32_t> tab;
  std::vector<int16_t> inv(2 * 729, -1);
  for (int q = 0; q < 2; ++q) {
    const int code = 9 - q;
    const double r = code / 2.0;
    std::vector<int32_t> main, extra;
    for (int dy = -4; dy <= 4; ++dy)
      for (int dx = -4; dx <= 4; ++dx) {
        const int d2 = dx * dx + dy * dy;
        if (4 * d2 > code * code) continue;
        const int zr = (int)std::floor(std::sqrt(r * r - d2) + 1e-12);
        main.push_back((int32_t)((uint32_t)(uint8_t)(int8_t)dx | ((uint32_t)(uint8_t)(int8_t)dy << 8) |
                                 ((uint32_t)zr << 16)));
      }
    if (code == 9) {
      // the last five single-node columns (zr = 0) are the extra columns of lanes 0..4, whose
      // own columns are the five shortest others (zr <= 1)
      for (int j = (int)main.size() - 1; j >= 0 && extra.size() < (size_t)(kColumns9 - 64); --j)
        if (((main[j] >> 16) & 255) == 0) {
          extra.insert(extra.begin(), main[j]);
          main.erase(main.begin() + j);
        }
      std::stable_sort(main.begin(), main.end(), [](int32_t a, int32_t b) { return ((a >> 16) & 255) < ((b >> 16) & 255); });
    }
    if (code == 9 && (main.size() != 64 || extra.size() != (size_t)(kColumns9 - 64))) {
      set_error("unexpected ball column count");
      return IB_ERR_ARG;
    }
    if (code == 8 && main.size() != (size_t)kColumns8) {
      set_error("unexpected ball column count");
      return IB_ERR_ARG;
    }
    tab.insert(tab.end(), main.begin(), main.end());
    tab.insert(tab.end(), extra.begin(), extra.end());
    const int st0 = w->balls.start[code], nb = w->balls.count[code];
    for (int b = 0; b < nb; ++b) {
      const uint32_t e = (uint32_t)w->balls.packed[st0 + b];
      const int dx = (int8_t)(e & 255), dy = (int8_t)((e >> 8) & 255), dz = (int8_t)((e >> 16) & 255);
      inv[q * 729 + ((dz + 4) * 9 + (dy + 4)) * 9 + (dx + 4)] = (int16_t)b;
    }
  }
  ib_status s;
  int16_t *d_inv = nullptr;
  int32_t *d_cnt = nullptr, *d_err = nullptr;
  auto cleanup = [&]() {
    dfree(d_inv);
    dfree(d_cnt);
    dfree(d_err);
  };
  if ((s = dalloc_t(&w->col_tab, tab.size())) || (s = dalloc_t(&w->zfirst, ncols)) || (s = dalloc_t(&d_inv, inv.size())) ||
      (s = dalloc_t(&d_cnt, nib)) || (s = dalloc_t(&w->col_off, nib)) || (s = dalloc_t(&d_err, 1))) {
    cleanup();
    return s;
  }
  IB_HIP(hipMemcpyAsync(w->col_tab, tab.data(), tab.size() * 4, hipMemcpyHostToDevice, st));
  IB_HIP(hipMemcpyAsync(d_inv, inv.data(), inv.size() * 2, hipMemcpyHostToDevice, st));
  IB_HIP(hipMemsetAsync(d_err, 0, 4, st));
  hipLaunchKernelGGL(k_zfirst, dim3((unsigned)((ncols + 255) / 256)), dim3(256), 0, st, w->node_class, (int)w->nx,
                     (int)w->ny, (int)w->nz, w->zfirst);
  hipLaunchKernelGGL(k_col_count, dim3((unsigned)nib), dim3(64), 0, st, nib, w->ib_xyz, w->zfirst, w->col_tab,
                     (int)w->nx, (int)w->ny, d_cnt);
  IB_HIP(hipGetLastError());
  std::vector<int32_t> cnt(nib);
  IB_HIP(hipMemcpyAsync(cnt.data(), d_cnt, nib * 4, hipMemcpyDeviceToHost, st));
  IB_HIP(hipStreamSynchronize(st));
  // the records start after kColPad entries: the tiled kernel's load windows reach up to 9
  // entries before a lane's first entry and up to 12 after it
  std::vector<uint32_t> off(nib, 0);
  int64_t tot = kColPad;
  for (int64_t i = 0; i < nib; ++i) {
    off[i] = (uint32_t)tot;
    if (cnt[i] > 0) tot += cnt[i];
  }
  if (tot >= (int64_t)UINT32_MAX) {
    cleanup();
    set_error("column-run stencil table too large");
    return IB_ERR_ARG;
  }
  if ((s = dalloc_t(&w->col32, tot + kColPad)) || (s = dalloc_t(&w->col64, tot + kColPad))) {
    cleanup();
    return s;
  }
  IB_HIP(hipMemsetAsync(w->col32, 0, (tot + kColPad) * sizeof(float), st));
  IB_HIP(hipMemsetAsync(w->col64, 0, (tot + kColPad) * sizeof(double), st));
  IB_HIP(hipMemcpyAsync(w->col_off, off.data(), nib * 4, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_col_pack, dim3((unsigned)nib), dim3(64), 0, st, nib, w->ib_xyz, w->ib_meta, w->rec32,
                     w->rec_off32, w->w64, w->zfirst, w->col_tab, d_inv, w->ball_meta, (int)w->nx, (int)w->ny,
                     (int)w->nz, w->col_off, d_cnt, w->col32, w->col64, d_err);
  IB_HIP(hipGetLastError());
  int32_t err = 0;
  IB_HIP(hipMemcpyAsync(&err, d_err, 4, hipMemcpyDeviceToHost, st));
  IB_HIP(hipStreamSynchronize(st));
  w->col_cnt = d_cnt;
  d_cnt = nullptr;
  cleanup();
  if (err) {
    set_error("column-run records: %d IB points have data nodes outside their runs", err);
    return IB_ERR_HIP;
  }
  w->col_words = tot + kColPad;
  w->stats.col_weights = tot - kColPad;
  return IB_OK;
}

ib_status weights_build(ib_weights *w, const int64_t *col_off_dev, hipStream_t st) {
  const int ndim = w->ndim, lat = ndim - 1, M = w->M;
  const int Kmax = w->prm.max_radius_steps;
  const int min_order = w->prm.min_basis_order;
  w->max_code = M + 1 + 2 * Kmax;
  ib_status s;
  if ((s = upload_ball_tables(w, st))) return s;

  const int64_t nib = w->nib;
  std::vector<int32_t> pending(nib);
  for (int64_t i = 0; i < nib; ++i) pending[i] = (int32_t)i;
  std::vector<int32_t> fin_k(nib, -1), fin_Mb(nib, 0), fin_nw(nib, 0), fin_round(nib, -1);
  std::vector<double> fin_sig(nib, 0.0);
  std::vector<RoundResult> rounds;
  int32_t *d_pending = nullptr, *d_status = nullptr, *d_ndata = nullptr, *desc = nullptr;
  double *d_sigma = nullptr, *bprel = nullptr;
  if ((s = dalloc_t(&d_pending, std::max<int64_t>(nib, 1))) || (s = dalloc_t(&d_status, std::max<int64_t>(nib, 1))) ||
      (s = dalloc_t(&d_ndata, std::max<int64_t>(nib, 1))) || (s = dalloc_t(&d_sigma, std::max<int64_t>(nib, 1))))
    return s;
  std::vector<int8_t> ex;
  multi_indices(M, ndim, ex);
  SolveConst sc{};
  for (size_t t = 0; t < ex.size() / 3; ++t)
    for (int q = 0; q < 3; ++q) sc.exps[t][q] = ex[t * 3 + q];
  second_derivative_weights(M, sc.w2);
  double max_cond = 0.0, min_margin = INFINITY;
  const double tol_base = 2.220446049250313e-16;
  // rows per streamed chunk: fewer, longer chunks halve the column steps of the 3D systems
  const int chunk = (ndim == 3) ? 64 : 48;
  // condition-value weights, kept on request: compacted per launch into device chunks,
  // concatenated at the end
  const bool keep_bc = w->prm.keep_bc_weights != 0;
  const int max_slots = keep_bc ? 8192 : 32768;
  struct BcChunk {
    int32_t *idx;
    double *w;
    int64_t n;
  };
  std::vector<BcChunk> bc_chunks;
  std::vector<int32_t> bc_chunk_of(keep_bc ? nib : 0, -1), bc_cnt(keep_bc ? nib : 0, 0);
  std::vector<int64_t> bc_loc(keep_bc ? nib : 0, 0);
  int32_t *d_fbp = nullptr, *d_fnbp = nullptr, *d_bpos = nullptr;
  double *d_fw = nullptr;
  int64_t *d_boff = nullptr;
  auto free_bc = [&]() {
    dfree(d_fbp), dfree(d_fnbp), dfree(d_bpos), dfree(d_fw), dfree(d_boff);
    d_fbp = d_fnbp = d_bpos = nullptr;
    d_fw = nullptr;
    d_boff = nullptr;
  };
  if (keep_bc && ((s = dalloc_t(&d_bpos, max_slots)) || (s = dalloc_t(&d_boff, max_slots)))) return s;

  for (int Mb = M; Mb >= min_order && !pending.empty(); --Mb) {
    const int NT = n_terms(Mb, ndim);
    sc.ops[0] = make_ops(w->prm.surface, Mb, ndim);
    IB_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(c_solve), &sc, sizeof(sc), 0, hipMemcpyHostToDevice, st));
    for (int k = 0; k <= Kmax && !pending.empty(); ++k) {
      const int code = Mb + 1 + 2 * k;
      const double r = code / 2.0;
      const int nball = w->balls.count[code];
      const int nwords = (nball + 31) / 32;
      const int maxbp = w->balls.count[std::min(code + 2, w->max_code + 2)] + 8;
      const int npend = (int)pending.size();
      RoundResult rr;
      rr.code = code;
      rr.k = k;
      rr.Mb = Mb;
      rr.nball = nball;
      rr.nwords = nwords;
      if ((s = dalloc_t(&rr.wout, (size_t)npend * nball)) || (s = dalloc_t(&rr.mout, (size_t)npend * nwords)))
        return s;
      IB_HIP(hipMemcpyAsync(d_pending, pending.data(), npend * 4, hipMemcpyHostToDevice, st));
      const int slots = std::min(npend, max_slots);
      const int desc_stride = nball;
      dfree(desc);
      dfree(bprel);
      if ((s = dalloc_t(&desc, (size_t)slots * desc_stride)) || (s = dalloc_t(&bprel, (size_t)slots * maxbp * 8)))
        return s;
      SolveArgs A{};
      A.cls = w->node_class;
      A.bp = w->bp;
      A.bpn = w->bp_normal;
      A.col_off = col_off_dev;
      A.ib_node = w->ib_node;
      A.nx = (int)w->nx;
      A.ny = (int)w->ny;
      A.nz = (int)w->nz;
      A.lat = lat;
      A.NT = NT;
      A.Mb = Mb;
      A.M = M;
      A.nops = sc.ops[0].nops;
      A.family = 0;
      A.gaxis = 0;
      A.nfields = 1;
      A.nblocks = 1;
      A.fcls[0] = w->node_class;
      A.fball[0] = w->ball + w->balls.start[code];
      A.fnball[0] = nball;
      A.fnwords[0] = nwords;
      A.fwoff[0] = 0;
      A.fblock[0] = 0;
      A.baxis[0] = 0;
      for (int q = 0; q < 3; ++q) {
        A.fshift[0][q] = 0.0;
        A.x0off[q] = 0.0;
      }
      A.xcls[0] = w->node_class;
      A.nball = nball;
      A.nwords = nwords;
      A.r2 = r * r;
      A.Rc = (int)floor(r + 0.5);
      A.rtol = w->prm.rank_rtol;
      A.robin_scale = (w->prm.physical_below ? -1.0 : 1.0) / w->h;
      A.chunk = chunk;
      A.desc = desc;
      A.desc_stride = desc_stride;
      A.bprel = bprel;
      A.maxbp = maxbp;
      A.wout = rr.wout;
      A.mout = rr.mout;
      A.status = d_status;
      A.ndata = d_ndata;
      A.sigma = d_sigma;
      if (keep_bc) {
        dfree(d_fbp), dfree(d_fw), dfree(d_fnbp);
        d_fbp = d_fnbp = nullptr;
        d_fw = nullptr;
        if ((s = dalloc_t(&d_fbp, (size_t)slots * maxbp)) || (s = dalloc_t(&d_fw, (size_t)slots * maxbp * A.nops)) ||
            (s = dalloc_t(&d_fnbp, slots)))
          return s;
        A.fbp = d_fbp;
        A.fwout = d_fw;
        A.fnbp = d_fnbp;
      }
      const int D1 = Mb + 1;
      size_t lds = sizeof(double) * ((size_t)NT * (NT + 1) / 2 + (size_t)chunk * 3 * D1 + (size_t)chunk * 3 +
                                     2 * (size_t)chunk + 4 + 2 * NT + 16) +
                   16 * sizeof(int);
      const void *kfn = (chunk == 64) ? (const void *)k_solve<64> : (const void *)k_solve<48>;
      IB_HIP(hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      const int sth = solve_threads(NT);
      for (int b0 = 0; b0 < npend; b0 += slots) {
        A.pending = d_pending + b0;
        A.npend = std::min(slots, npend - b0);
        A.out_base = b0;
        if (chunk == 64)
          hipLaunchKernelGGL(k_solve<64>, dim3(A.npend), dim3(sth), lds, st, A);
        else
          hipLaunchKernelGGL(k_solve<48>, dim3(A.npend), dim3(sth), lds, st, A);
        IB_HIP(hipGetLastError());
        if (keep_bc) {
          // compact this launch's condition-value weights of the accepted points
          const int nl = A.npend;
          std::vector<int32_t> ls(nl), lf(nl), apos;
          std::vector<int64_t> aoff;
          IB_HIP(hipMemcpyAsync(ls.data(), d_status + b0, nl * 4, hipMemcpyDeviceToHost, st));
          IB_HIP(hipMemcpyAsync(lf.data(), d_fnbp, nl * 4, hipMemcpyDeviceToHost, st));
          IB_HIP(hipStreamSynchronize(st));
          int64_t tot = 0;
          for (int q = 0; q < nl; ++q) {
            if (ls[q] != 1) continue;
            const int id = pending[b0 + q];
            apos.push_back(q);
            aoff.push_back(tot);
            bc_chunk_of[id] = (int32_t)bc_chunks.size();
            bc_loc[id] = tot;
            bc_cnt[id] = lf[q] * A.nops;
            tot += (int64_t)lf[q] * A.nops;
          }
          BcChunk c{nullptr, nullptr, tot};
          if ((s = dalloc_t(&c.idx, std::max<int64_t>(tot, 1))) || (s = dalloc_t(&c.w, std::max<int64_t>(tot, 1))))
            return s;
          bc_chunks.push_back(c);
          if (!apos.empty()) {
            IB_HIP(hipMemcpyAsync(d_bpos, apos.data(), apos.size() * 4, hipMemcpyHostToDevice, st));
            IB_HIP(hipMemcpyAsync(d_boff, aoff.data(), aoff.size() * 8, hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL(k_pack_bc, dim3((unsigned)apos.size()), dim3(256), 0, st, (int)apos.size(), d_bpos,
                               d_boff, d_fbp, d_fw, d_fnbp, maxbp, A.nops, c.idx, c.w);
            IB_HIP(hipGetLastError());
            IB_HIP(hipStreamSynchronize(st));
          }
        }
      }
      std::vector<int32_t> hs(npend), hn(npend);
      std::vector<double> hsig(npend);
      IB_HIP(hipMemcpyAsync(hs.data(), d_status, npend * 4, hipMemcpyDeviceToHost, st));
      IB_HIP(hipMemcpyAsync(hn.data(), d_ndata, npend * 4, hipMemcpyDeviceToHost, st));
      IB_HIP(hipMemcpyAsync(hsig.data(), d_sigma, npend * 8, hipMemcpyDeviceToHost, st));
      IB_HIP(hipStreamSynchronize(st));
      std::vector<int32_t> next;
      for (int p = 0; p < npend; ++p) {
        int id = pending[p];
        if (hs[p] < 0) {
          set_error("IB point %d: support scratch overflow (radius %.1f)", id, r);
          return IB_ERR_ARG;
        }
        if (hs[p] == 1) {
          fin_k[id] = k;
          fin_Mb[id] = Mb;
          fin_nw[id] = hn[p];
          fin_round[id] = (int)rounds.size();
          fin_sig[id] = hsig[p];
          rr.acc_pos.push_back(p);
          rr.acc_id.push_back(id);
          max_cond = std::max(max_cond, 1.0 / hsig[p]);
          (void)tol_base;
        } else {
          next.push_back(id);
        }
      }
      rounds.push_back(std::move(rr));
      pending.swap(next);
    }
  }
  dfree(desc);
  dfree(bprel);
  dfree(d_pending);
  dfree(d_status);
  dfree(d_ndata);
  free_bc();
  if (!pending.empty()) {
    dfree(d_sigma);
    for (auto &rr : rounds) dfree(rr.wout), dfree(rr.mout);
    for (auto &c : bc_chunks) dfree(c.idx), dfree(c.w);
    set_error("%zu IB points remain rank deficient after radius growth and order reduction (first: node %d)",
              pending.size(), pending[0]);
    return IB_ERR_UNCONSTRAINED;
  }
  // offsets and final tables
  std::vector<int32_t> woff(nib);
  std::vector<uint32_t> roff32(nib), roff64(nib);
  std::vector<int16_t> xyz(nib * 4);
  std::vector<int32_t> meta(nib * 4);
  std::vector<int64_t> hnode(nib);
  IB_HIP(hipMemcpyAsync(hnode.data(), w->ib_node, nib * 8, hipMemcpyDeviceToHost, st));
  IB_HIP(hipStreamSynchronize(st));
  int64_t sw = 0, s32 = 0, s64 = 0;
  int64_t maxnw = 0;
  for (int64_t i = 0; i < nib; ++i) {
    const RoundResult &rr = rounds[fin_round[i]];
    woff[i] = (int32_t)sw;
    roff32[i] = (uint32_t)s32;
    roff64[i] = (uint32_t)s64;
    sw += fin_nw[i];
    s32 += rr.nwords + fin_nw[i];
    s64 += ((rr.nwords + 1) & ~1) + 2 * (int64_t)fin_nw[i];
    maxnw = std::max<int64_t>(maxnw, fin_nw[i]);
    int64_t nd = hnode[i];
    xyz[i * 4 + 0] = (int16_t)(nd % w->nx);
    xyz[i * 4 + 1] = (int16_t)((nd / w->nx) % w->ny);
    xyz[i * 4 + 2] = (int16_t)(nd / (w->nx * w->ny));
    xyz[i * 4 + 3] = (int16_t)rr.code;
    meta[i * 4 + 0] = fin_k[i];
    meta[i * 4 + 1] = fin_Mb[i];
    meta[i * 4 + 2] = fin_nw[i];
    meta[i * 4 + 3] = woff[i];
    w->stats.radius_hist[std::min(fin_k[i], 7)]++;
    w->stats.order_hist[std::min(fin_Mb[i], 16)]++;
    min_margin = std::min(min_margin, fin_sig[i] / (std::max<double>(fin_nw[i], 1) * tol_base));
  }
  if (s32 >= (int64_t)UINT32_MAX || s64 >= (int64_t)UINT32_MAX || sw >= (int64_t)INT32_MAX) {
    set_error("stencil table too large (%lld weights)", (long long)sw);
    return IB_ERR_ARG;
  }
  w->sumw = sw;
  w->rec32_words = s32;
  w->rec64_words = s64;
  w->stats.sum_nw = sw;
  w->stats.max_nw = maxnw;
  w->stats.max_cond = max_cond;
  w->stats.min_margin = min_margin;
  w->stats.table_bytes_f32 = s32 * 4;
  w->stats.table_bytes_f64 = s64 * 4;
  if ((s = dalloc_t(&w->w64, std::max<int64_t>(sw, 1))) || (s = dalloc_t(&w->rec32, std::max<int64_t>(s32, 1))) ||
      (s = dalloc_t(&w->rec64, std::max<int64_t>(s64, 1))) || (s = dalloc_t(&w->rec_off32, std::max<int64_t>(nib, 1))) ||
      (s = dalloc_t(&w->rec_off64, std::max<int64_t>(nib, 1))) || (s = dalloc_t(&w->ib_xyz, std::max<int64_t>(nib, 1) * 4)) ||
      (s = dalloc_t(&w->ib_meta, std::max<int64_t>(nib, 1) * 4)) || (s = dalloc_t(&w->ib_sigma, std::max<int64_t>(nib, 1))))
    return s;
  int32_t *d_woff = nullptr, *d_nw = nullptr, *d_apos = nullptr, *d_aid = nullptr;
  if ((s = dalloc_t(&d_woff, std::max<int64_t>(nib, 1))) || (s = dalloc_t(&d_nw, std::max<int64_t>(nib, 1))) ||
      (s = dalloc_t(&d_apos, std::max<int64_t>(nib, 1))) || (s = dalloc_t(&d_aid, std::max<int64_t>(nib, 1))))
    return s;
  IB_HIP(hipMemcpyAsync(d_woff, woff.data(), nib * 4, hipMemcpyHostToDevice, st));
  IB_HIP(hipMemcpyAsync(d_nw, fin_nw.data(), nib * 4, hipMemcpyHostToDevice, st));
  IB_HIP(hipMemcpyAsync(w->rec_off32, roff32.data(), nib * 4, hipMemcpyHostToDevice, st));
  IB_HIP(hipMemcpyAsync(w->rec_off64, roff64.data(), nib * 4, hipMemcpyHostToDevice, st));
  IB_HIP(hipMemcpyAsync(w->ib_xyz, xyz.data(), nib * 8, hipMemcpyHostToDevice, st));
  IB_HIP(hipMemcpyAsync(w->ib_meta, meta.data(), nib * 16, hipMemcpyHostToDevice, st));
  IB_HIP(hipMemcpyAsync(w->ib_sigma, fin_sig.data(), nib * 8, hipMemcpyHostToDevice, st));
  for (auto &rr : rounds) {
    int nacc = (int)rr.acc_pos.size();
    if (nacc) {
      IB_HIP(hipMemcpyAsync(d_apos, rr.acc_pos.data(), nacc * 4, hipMemcpyHostToDevice, st));
      IB_HIP(hipMemcpyAsync(d_aid, rr.acc_id.data(), nacc * 4, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_pack, dim3(nacc), dim3(256), 0, st, nacc, d_apos, d_aid, rr.wout, rr.nball, rr.mout,
                         rr.nwords, d_woff, d_nw, w->rec_off32, w->rec_off64, w->w64, w->rec32, w->rec64);
      IB_HIP(hipGetLastError());
      IB_HIP(hipStreamSynchronize(st));
    }
    dfree(rr.wout);
    dfree(rr.mout);
    w->stats.max_ball = std::max<int64_t>(w->stats.max_ball, rr.nball);
  }
  IB_HIP(hipStreamSynchronize(st));
  dfree(d_woff), dfree(d_nw), dfree(d_apos), dfree(d_aid), dfree(d_sigma);
  if (keep_bc) {
    std::vector<int64_t> base(bc_chunks.size() + 1, 0);
    for (size_t c = 0; c < bc_chunks.size(); ++c) base[c + 1] = base[c] + bc_chunks[c].n;
    const int64_t nbc = base.back();
    if ((s = dalloc_t(&w->bc_idx, std::max<int64_t>(nbc, 1))) || (s = dalloc_t(&w->bc_w, std::max<int64_t>(nbc, 1))) ||
        (s = dalloc_t(&w->bc_off, std::max<int64_t>(nib, 1))) || (s = dalloc_t(&w->bc_cnt, std::max<int64_t>(nib, 1))))
      return s;
    for (size_t c = 0; c < bc_chunks.size(); ++c) {
      if (bc_chunks[c].n) {
        IB_HIP(hipMemcpyAsync(w->bc_idx + base[c], bc_chunks[c].idx, bc_chunks[c].n * 4, hipMemcpyDeviceToDevice, st));
        IB_HIP(hipMemcpyAsync(w->bc_w + base[c], bc_chunks[c].w, bc_chunks[c].n * 8, hipMemcpyDeviceToDevice, st));
      }
    }
    std::vector<int64_t> off(nib);
    for (int64_t i = 0; i < nib; ++i) off[i] = base[bc_chunk_of[i]] + bc_loc[i];
    IB_HIP(hipMemcpyAsync(w->bc_off, off.data(), nib * 8, hipMemcpyHostToDevice, st));
    IB_HIP(hipMemcpyAsync(w->bc_cnt, bc_cnt.data(), nib * 4, hipMemcpyHostToDevice, st));
    IB_HIP(hipStreamSynchronize(st));
    for (auto &c : bc_chunks) dfree(c.idx), dfree(c.w);
    w->nbc = nbc;
    w->bc_nq = make_ops(w->prm.surface, M, ndim).nops;
  }
  if ((s = build_dense_records(w, st))) return s;
  return build_column_records(w, st);
}

// Batched solves of one family of staggered operators (first-order form): the same
// kernel as the pressure form, with the family's data fields, half-cell supports,
// expansion point and coupled unknown blocks; results come back to the host.
ib_status solve_family(ib_weights *w, const FamilySpec &F, const int64_t *col_off_dev, hipStream_t st,
                       std::vector<FamilyPoint> &out) {
  const int ndim = w->ndim, lat = ndim - 1, M = w->M;
  const int Kmax = w->prm.max_radius_steps, min_order = w->prm.min_basis_order;
  const int64_t np = (int64_t)F.anchors.size();
  out.assign(np, FamilyPoint());
  if (np == 0) return IB_OK;
  ib_status s;
  int64_t *d_anchor = nullptr;
  int32_t *d_pending = nullptr, *d_status = nullptr, *d_ndata = nullptr;
  double *d_sigma = nullptr;
  if ((s = dalloc_t(&d_anchor, np)) || (s = dalloc_t(&d_pending, np)) || (s = dalloc_t(&d_status, np)) ||
      (s = dalloc_t(&d_ndata, np)) || (s = dalloc_t(&d_sigma, np)))
    return s;
  IB_HIP(hipMemcpy(d_anchor, F.anchors.data(), np * 8, hipMemcpyHostToDevice));
  std::vector<int32_t> pending(np);
  for (int64_t i = 0; i < np; ++i) pending[i] = (int32_t)i;
  std::vector<int8_t> ex;
  multi_indices(M, ndim, ex);
  SolveConst sc;
  std::memset(&sc, 0, sizeof(sc));
  for (size_t t = 0; t < ex.size() / 3; ++t)
    for (int q = 0; q < 3; ++q) sc.exps[t][q] = ex[t * 3 + q];
  second_derivative_weights(M, sc.w2);
  staggered_first_derivative_weights(M, sc.ws);
  const int chunk = (ndim == 3) ? 32 : 48;
  const int max_slots = 32768;
  for (int Mb = M; Mb >= min_order && !pending.empty(); --Mb) {
    const int NT = n_terms(Mb, ndim), NTT = NT * F.nblocks;
    if (NTT > 192) {
      set_error("staggered velocity system of %d unknowns exceeds the solver's 192", NTT);
      return IB_ERR_ARG;
    }
    for (int b = 0; b < F.nblocks; ++b)
      sc.ops[b] = (F.family == 1) ? make_ops(w->prm.surface, Mb, ndim) : make_vops(w->prm.surface, Mb, ndim, F.baxis[b]);
    IB_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(c_solve), &sc, sizeof(sc), 0, hipMemcpyHostToDevice, st));
    for (int k = 0; k <= Kmax && !pending.empty(); ++k) {
      const int code = Mb + 1 + 2 * k;
      const double r = code / 2.0;
      // shifted lattice balls of the data fields
      std::vector<int32_t> tab;
      int fstart[3] = {0, 0, 0}, fnb[3] = {0, 0, 0}, fnw[3] = {0, 0, 0}, fwo[3] = {0, 0, 0};
      int nball = 0, nwords = 0;
      double shift[3][3];
      for (int f = 0; f < F.nfields; ++f) {
        for (int q = 0; q < 3; ++q) shift[f][q] = F.foff[f][q] - F.x0off[q];
        std::vector<int32_t> b = shifted_ball(ndim, code, shift[f]);
        fstart[f] = (int)tab.size();
        fnb[f] = (int)b.size();
        fnw[f] = (fnb[f] + 31) / 32;
        fwo[f] = nwords;
        nball += fnb[f];
        nwords += fnw[f];
        tab.insert(tab.end(), b.begin(), b.end());
      }
      int32_t *d_tab = nullptr, *desc = nullptr;
      double *bprel = nullptr, *wout = nullptr;
      uint32_t *mout = nullptr;
      const int npend = (int)pending.size();
      const int slots = std::min(npend, max_slots);
      BallTables bt;
      bt.build(ndim, code + 2);
      const int maxbp = bt.count[code + 2] + 8;
      if ((s = dalloc_t(&d_tab, tab.size())) || (s = dalloc_t(&desc, (size_t)slots * nball)) ||
          (s = dalloc_t(&bprel, (size_t)slots * maxbp * 8)) || (s = dalloc_t(&wout, (size_t)npend * nball)) ||
          (s = dalloc_t(&mout, (size_t)npend * nwords)))
        return s;
      IB_HIP(hipMemcpy(d_tab, tab.data(), tab.size() * 4, hipMemcpyHostToDevice));
      IB_HIP(hipMemcpyAsync(d_pending, pending.data(), npend * 4, hipMemcpyHostToDevice, st));
      SolveArgs A{};
      A.family = F.family;
      A.gaxis = F.gaxis;
      A.nfields = F.nfields;
      A.nblocks = F.nblocks;
      for (int f = 0; f < 3; ++f) {
        A.fcls[f] = F.fcls[f];
        A.fball[f] = d_tab + fstart[f];
        A.fnball[f] = fnb[f];
        A.fnwords[f] = fnw[f];
        A.fwoff[f] = fwo[f];
        for (int q = 0; q < 3; ++q) A.fshift[f][q] = (f < F.nfields) ? shift[f][q] : 0.0;
        A.fblock[f] = F.fblock[f];
        A.baxis[f] = F.baxis[f];
        A.xcls[f] = F.xcls[f];
        A.x0off[f] = F.x0off[f];
      }
      A.cls = w->node_class;
      A.bp = w->bp;
      A.bpn = w->bp_normal;
      A.col_off = col_off_dev;
      A.ib_node = d_anchor;
      A.nx = (int)w->nx;
      A.ny = (int)w->ny;
      A.nz = (int)w->nz;
      A.lat = lat;
      A.NT = NT;
      A.Mb = Mb;
      A.M = M;
      A.nops = sc.ops[0].nops;
      A.nball = nball;
      A.nwords = nwords;
      A.r2 = r * r;
      A.Rc = (int)floor(r + 1.0);
      A.rtol = w->prm.rank_rtol;
      A.chunk = chunk;
      A.desc = desc;
      A.desc_stride = nball;
      A.bprel = bprel;
      A.maxbp = maxbp;
      A.wout = wout;
      A.mout = mout;
      A.status = d_status;
      A.ndata = d_ndata;
      A.sigma = d_sigma;
      const int D1 = Mb + 1;
      size_t lds = sizeof(double) * ((size_t)NTT * (NTT + 1) / 2 + (size_t)chunk * 3 * D1 + (size_t)chunk * 3 +
                                     2 * (size_t)chunk + 4 + 2 * NTT + 16) +
                   16 * sizeof(int);
      const void *kfn = (chunk == 32) ? (const void *)k_solve<32> : (const void *)k_solve<48>;
      IB_HIP(hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      const int sth = solve_threads(NTT);
      for (int b0 = 0; b0 < npend; b0 += slots) {
        A.pending = d_pending + b0;
        A.npend = std::min(slots, npend - b0);
        A.out_base = b0;
        if (chunk == 32)
          hipLaunchKernelGGL(k_solve<32>, dim3(A.npend), dim3(sth), lds, st, A);
        else
          hipLaunchKernelGGL(k_solve<48>, dim3(A.npend), dim3(sth), lds, st, A);
        IB_HIP(hipGetLastError());
      }
      std::vector<int32_t> hs(npend), hn(npend);
      std::vector<double> hw((size_t)npend * nball);
      std::vector<uint32_t> hm((size_t)npend * nwords);
      IB_HIP(hipMemcpyAsync(hs.data(), d_status, npend * 4, hipMemcpyDeviceToHost, st));
      IB_HIP(hipMemcpyAsync(hn.data(), d_ndata, npend * 4, hipMemcpyDeviceToHost, st));
      IB_HIP(hipMemcpyAsync(hw.data(), wout, hw.size() * 8, hipMemcpyDeviceToHost, st));
      IB_HIP(hipMemcpyAsync(hm.data(), mout, hm.size() * 4, hipMemcpyDeviceToHost, st));
      IB_HIP(hipStreamSynchronize(st));
      std::vector<int32_t> next;
      for (int p = 0; p < npend; ++p) {
        const int id = pending[p];
        if (hs[p] < 0) {
          set_error("staggered family %d point %d: support scratch overflow (radius %.1f)", F.family, id, r);
          return IB_ERR_ARG;
        }
        if (hs[p] != 1) {
          next.push_back(id);
          continue;
        }
        FamilyPoint &fp = out[id];
        fp.k = k;
        fp.Mb = Mb;
        int kk = 0;
        for (int f = 0; f < F.nfields; ++f) {
          const uint32_t *m = hm.data() + (size_t)p * nwords + fwo[f];
          for (int b = 0; b < fnb[f]; ++b) {
            if (!((m[b >> 5] >> (b & 31)) & 1u)) continue;
            fp.field.push_back(f);
            fp.off.push_back(tab[fstart[f] + b]);
            fp.w.push_back(hw[(size_t)p * nball + kk]);
            ++kk;
          }
        }
        if (kk != hn[p]) {
          set_error("staggered family %d point %d: mask/weight count mismatch", F.family, id);
          return IB_ERR_HIP;
        }
      }
      dfree(d_tab), dfree(desc), dfree(bprel), dfree(wout), dfree(mout);
      pending.swap(next);
    }
  }
  dfree(d_anchor), dfree(d_pending), dfree(d_status), dfree(d_ndata), dfree(d_sigma);
  if (!pending.empty()) {
    set_error("%zu staggered-family points remain rank deficient (family %d)", pending.size(), F.family);
    return IB_ERR_UNCONSTRAINED;
  }
  return IB_OK;
}

}  // namespace ib
