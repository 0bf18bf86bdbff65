// Shared host-side helpers: error reporting, allocation, lattice balls, operator tables.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <utility>

#include "ib_internal.h"

namespace ib {

static thread_local std::string g_err;

const char *last_error_text() { return g_err.c_str(); }

void set_error(const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}

ib_status hip_fail(hipError_t e, const char *what, const char *file, int line) {
  set_error("%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  return (e == hipErrorOutOfMemory) ? IB_ERR_OOM : IB_ERR_HIP;
}

ib_status dalloc(void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    *p = nullptr;
    return IB_ERR_OOM;
  }
  return IB_OK;
}

void dfree(void *p) {
  if (p) (void)hipFree(p);
}

void BallTables::build(int ndim, int max_code) {
  packed.clear();
  for (int c = 1; c <= max_code; ++c) {
    start[c] = (int)packed.size();
    int R = c / 2;
    long long r2x4 = (long long)c * c;   // (2r)^2; |o|^2 <= r^2  <=>  4|o|^2 <= (2r)^2
    int zlo = -R, zhi = R, ylo = (ndim == 3) ? -R : 0, yhi = (ndim == 3) ? R : 0;
    for (int dz = zlo; dz <= zhi; ++dz)
      for (int dy = ylo; dy <= yhi; ++dy)
        for (int dx = -R; dx <= R; ++dx) {
          long long s = 4LL * (dx * dx + dy * dy + dz * dz);
          if (s <= r2x4) {
            uint32_t v = (uint32_t)(uint8_t)(int8_t)dx | ((uint32_t)(uint8_t)(int8_t)dy << 8) |
                         ((uint32_t)(uint8_t)(int8_t)dz << 16);
            packed.push_back((int32_t)v);
          }
        }
    count[c] = (int)packed.size() - start[c];
  }
}

int n_terms(int M, int ndim) {
  long long n = 1;
  for (int i = 1; i <= ndim; ++i) n = n * (M + i) / i;
  return (int)n;
}

// Graded order: degree 0..M; inside a degree the x exponent descends, then y.
void multi_indices(int M, int ndim, std::vector<int8_t> &out) {
  out.clear();
  for (int k = 0; k <= M; ++k) {
    if (ndim == 2) {
      for (int a = k; a >= 0; --a) {
        out.push_back((int8_t)a);
        out.push_back(0);
        out.push_back((int8_t)(k - a));
      }
    } else {
      for (int a = k; a >= 0; --a)
        for (int b = k - a; b >= 0; --b) {
          out.push_back((int8_t)a);
          out.push_back((int8_t)b);
          out.push_back((int8_t)(k - a - b));
        }
    }
  }
}

// Centred second-derivative weights of order M = 2m (grid units), closed form
// w_k = 2 (-1)^(k+1) (m!)^2 / (k^2 (m-k)! (m+k)!), w_0 = -2 sum_k w_k.
void second_derivative_weights(int M, double *w) {
  int m = M / 2;
  auto fact = [](int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
  };
  double s = 0.0;
  for (int k = 1; k <= m; ++k) {
    double v = 2.0 * ((k % 2) ? 1.0 : -1.0) * fact(m) * fact(m) / ((double)k * k * fact(m - k) * fact(m + k));
    w[m + k] = v;
    w[m - k] = v;
    s += v;
  }
  w[m] = -2.0 * s;
}

// Staggered first derivative at 0 from M nodes at offsets -(M-1)/2 .. (M-1)/2: the
// weights make sum_k w_k x_k^j equal to the j-th derivative of x^j at 0 (1 for j = 1,
// else 0) for j < M; solved by Gaussian elimination with partial pivoting (M <= 8).
void staggered_first_derivative_weights(int M, double *w) {
  double A[kMaxOrder][kMaxOrder + 1];
  for (int j = 0; j < M; ++j) {
    for (int k = 0; k < M; ++k) A[j][k] = std::pow(k - (M - 1) / 2.0, j);
    A[j][M] = (j == 1) ? 1.0 : 0.0;
  }
  for (int c = 0; c < M; ++c) {
    int piv = c;
    for (int r = c + 1; r < M; ++r)
      if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
    for (int k = 0; k <= M; ++k) std::swap(A[c][k], A[piv][k]);
    for (int r = 0; r < M; ++r) {
      if (r == c) continue;
      const double f = A[r][c] / A[c][c];
      for (int k = c; k <= M; ++k) A[r][k] -= f * A[c][k];
    }
  }
  for (int k = 0; k < M; ++k) w[k] = A[k][M] / A[k][k];
}

// nabla^{2q} in d dimensions: sum over |g| = q of q!/g! d^{2g}.
void add_laplacian_power(OpSet &ops, int slot, int q, int ndim, int normal_axis, int scaled) {
  auto fact = [](int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
  };
  for (int a = q; a >= 0; --a) {
    for (int b = (ndim == 3 ? q - a : 0); b >= 0; --b) {
      int c = q - a - b;
      if (ndim == 2) {
        c = q - a;
        b = 0;
      }
      double coef = fact(q) / (fact(a) * fact(b) * fact(c));
      OpTerm t{};
      t.beta[0] = (int8_t)(2 * a);
      t.beta[1] = (int8_t)(2 * b);
      t.beta[2] = (int8_t)(2 * c);
      t.normal_axis = (int8_t)normal_axis;
      t.scaled = (int8_t)scaled;
      t.coef = coef;
      if (normal_axis >= 0) t.beta[normal_axis] += 1;
      ops.term[slot][ops.nterms[slot]++] = t;
      if (ndim == 2) break;
    }
  }
}

OpSet make_ops(int surface, int Mb, int ndim) {
  OpSet ops;
  memset(&ops, 0, sizeof(ops));
  if (surface == IB_SURF_FREE) {
    for (int q = 0; 2 * q <= Mb; ++q) {
      add_laplacian_power(ops, ops.nops, q, ndim, -1);
      ops.nops++;
    }
  } else if (surface == IB_SURF_ROBIN) {
    // (1 + a n_out . grad) nabla^{2q} for 2q <= Mb (the free-surface members; none reduces
    // to 0 = 0 on the basis); the normal part of order 2q + 1 > Mb vanishes on the basis and
    // is left out.  The sign of n_out relative to the stored normal is folded into the
    // per-point coefficient.
    for (int q = 0; 2 * q <= Mb; ++q) {
      add_laplacian_power(ops, ops.nops, q, ndim, -1);
      for (int ax = 0; ax < 3 && 2 * q + 1 <= Mb; ++ax) {
        if (ndim == 2 && ax == 1) continue;
        add_laplacian_power(ops, ops.nops, q, ndim, ax, 1);
      }
      ops.nops++;
    }
  } else {
    for (int q = 0; 2 * q + 1 <= Mb; ++q) {
      // n . grad (nabla^{2q}): the lateral axes then depth (2D uses axes x and z)
      for (int ax = 0; ax < 3; ++ax) {
        if (ndim == 2 && ax == 1) continue;
        add_laplacian_power(ops, ops.nops, q, ndim, ax);
      }
      ops.nops++;
    }
  }
  return ops;
}

// Velocity rows of the first-order form, block ``axis`` (the v_axis component):
//   free:  lap^q (div v) = 0 for 2q+1 <= Mb  ->  d_axis lap^q on this block;
//   rigid: n.v = 0 (normal component on this block), then n.grad lap^(q-1) div v = 0
//          for 2q <= Mb  ->  n.grad lap^(q-1) d_axis on this block.
OpSet make_vops(int surface, int Mb, int ndim, int axis) {
  OpSet ops;
  memset(&ops, 0, sizeof(ops));
  auto shift_slot = [&](int slot, int ax) {
    for (int t = 0; t < ops.nterms[slot]; ++t) ops.term[slot][t].beta[ax] += 1;
  };
  if (surface == IB_SURF_FREE) {
    for (int q = 0; 2 * q + 1 <= Mb; ++q) {
      add_laplacian_power(ops, ops.nops, q, ndim, -1);
      shift_slot(ops.nops, axis);
      ops.nops++;
    }
  } else {
    OpTerm t{};
    t.normal_axis = (int8_t)axis;
    t.coef = 1.0;
    ops.term[0][0] = t;
    ops.nterms[0] = 1;
    ops.nops = 1;
    for (int q = 1; 2 * q <= Mb; ++q) {
      for (int ax = 0; ax < 3; ++ax) {
        if (ndim == 2 && ax == 1) continue;
        const int before = ops.nterms[ops.nops];
        add_laplacian_power(ops, ops.nops, q - 1, ndim, ax);
        for (int k = before; k < ops.nterms[ops.nops]; ++k) ops.term[ops.nops][k].beta[axis] += 1;
      }
      ops.nops++;
    }
  }
  return ops;
}

// Lattice points o with |o + shift| <= r (r = code / 2) in memory order, packed like the
// canonical balls.  shift components are multiples of 1/2.
std::vector<int32_t> shifted_ball(int ndim, int code, const double shift[3]) {
  std::vector<int32_t> out;
  const double r = code / 2.0;
  const int R = (int)std::floor(r) + 1;
  const int ylo = (ndim == 3) ? -R : 0, yhi = (ndim == 3) ? R : 0;
  for (int dz = -R; dz <= R; ++dz)
    for (int dy = ylo; dy <= yhi; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        const double ax = dx + shift[0], ay = dy + shift[1], az = dz + shift[2];
        if (ax * ax + ay * ay + az * az <= r * r) {
          uint32_t v = (uint32_t)(uint8_t)(int8_t)dx | ((uint32_t)(uint8_t)(int8_t)dy << 8) |
                       ((uint32_t)(uint8_t)(int8_t)dz << 16);
          out.push_back((int32_t)v);
        }
      }
  return out;
}

}  // namespace ib
