// HIP kernels of the H-LU library (gfx950).
//
// Every kernel of the factorisation schedule processes one descriptor per
// workgroup (256 threads = four 64-wide wavefronts); a launch covers one
// batch (all descriptors of one type in one wave of the schedule).  Small
// tiles are staged through LDS; low-rank panels are streamed in row chunks.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ops.h"

namespace hlu {

#define NT 256

// live column count: ranks change while a schedule runs, so they are read
// with a device-scope atomic load (never through a cached scalar load)
__device__ __forceinline__ int pcols(const PRef& r) {
  return r.rankp ? __hip_atomic_load(reinterpret_cast<int32_t*>(r.rankp), __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT)
                 : r.cols;
}

__device__ __forceinline__ double pget(const PRef& r, int i, int j) {
  if (r.kind == PK_IDENT) return (j == i + r.ld) ? 1.0 : 0.0;
  size_t k = r.trans ? (size_t)j + (size_t)i * r.ld : (size_t)i + (size_t)j * r.ld;
  return r.dt == DT_F64 ? reinterpret_cast<const double*>(r.ptr)[k]
                        : (double)reinterpret_cast<const float*>(r.ptr)[k];
}

__device__ __forceinline__ void pset(const PRef& r, int i, int j, double v) {
  size_t k = r.trans ? (size_t)j + (size_t)i * r.ld : (size_t)i + (size_t)j * r.ld;
  if (r.dt == DT_F64) reinterpret_cast<double*>(r.ptr)[k] = v;
  else reinterpret_cast<float*>(r.ptr)[k] = (float)v;
}

// per-op record {model flops, algorithmic bytes, rank-capacity hit, rank,
// start tick, end tick, stack width, 0} (ticks of the constant-rate wall
// clock, written by thread 0)
__device__ __forceinline__ void put_cost(const Op& op, double flops, double bytes,
                                         double cap_hit = 0.0, double rank = 0.0,
                                         double width = 0.0) {
  if (op.cost && threadIdx.x == 0) {
    double* c = reinterpret_cast<double*>(op.cost);
    c[0] = flops;
    c[1] = bytes;
    c[2] = cap_hit;
    c[3] = rank;
    c[5] = (double)wall_clock64();
    c[6] = width;
  }
}

__device__ __forceinline__ void start_tick(const Op& op) {
  if (op.cost && threadIdx.x == 0) reinterpret_cast<double*>(op.cost)[4] = (double)wall_clock64();
}

// ---------------------------------------------------------------- getrf
// Right-looking unblocked LU with partial pivoting of one b x b leaf
// (b <= 64) held in LDS; pivot = first row of the largest |a_ik|.
// Contraction is disabled so that the elimination rounds exactly like the
// textbook update a - l*u.
#define LDS_GETRF (64 * 65 * 8 + 16)
__device__ void d_getrf(const Op& op, char* smem) {
#pragma clang fp contract(off)
  const PRef A = op.p[0];
  const int b = A.rows;
  double (*a)[65] = reinterpret_cast<double (*)[65]>(smem);
  int& s_piv = reinterpret_cast<int*>(smem + 64 * 65 * 8)[0];
  int& s_info = reinterpret_cast<int*>(smem + 64 * 65 * 8)[1];
  const int tid = threadIdx.x;
  double* g = reinterpret_cast<double*>(A.ptr);
  for (int e = tid; e < b * b; e += NT) {
    int i = e % b, j = e / b;
    a[i][j] = g[i + (size_t)j * A.ld];
  }
  if (tid == 0) s_info = 0;
  int32_t* piv = reinterpret_cast<int32_t*>(op.p[1].ptr);
  __syncthreads();
  for (int k = 0; k < b; ++k) {
    if (tid < 64) {
      double v = (tid >= k && tid < b) ? fabs(a[tid][k]) : -1.0;
      int ix = tid;
      for (int o = 32; o > 0; o >>= 1) {
        double v2 = __shfl_xor(v, o);
        int i2 = __shfl_xor(ix, o);
        if (v2 > v || (v2 == v && i2 < ix)) { v = v2; ix = i2; }
      }
      if (tid == 0) {
        s_piv = ix;
        piv[k] = ix;
        if (a[ix][k] == 0.0 && s_info == 0) s_info = k + 1;
      }
    }
    __syncthreads();
    const int p = s_piv;
    const bool nz = a[p][k] != 0.0;
    if (nz && p != k) {
      for (int j = tid; j < b; j += NT) {
        double t = a[k][j];
        a[k][j] = a[p][j];
        a[p][j] = t;
      }
    }
    __syncthreads();
    if (nz) {
      const double d = a[k][k];
      for (int i = k + 1 + tid; i < b; i += NT) a[i][k] = a[i][k] / d;
    }
    __syncthreads();
    const int r = b - k - 1;
    for (int e = tid; e < r * r; e += NT) {
      int i = k + 1 + e % r, j = k + 1 + e / r;
      double prod = a[i][k] * a[k][j];
      a[i][j] = a[i][j] - prod;
    }
    __syncthreads();
  }
  for (int e = tid; e < b * b; e += NT) {
    int i = e % b, j = e / b;
    g[i + (size_t)j * A.ld] = a[i][j];
  }
  if (tid == 0 && s_info != 0 && op.p[1].rankp) {
    int32_t* st = reinterpret_cast<int32_t*>(op.p[1].rankp);
    atomicCAS(st, 0, op.i0 + s_info);
  }
  put_cost(op, 2.0 * b * b * b / 3.0 - b * b / 2.0 + 5.0 * b / 6.0, 16.0 * b * b);
}

// ---------------------------------------------------------------- leaf solves
// p1 := L^{-1} P p1 (OP_TRSM_L), U^{-T} p1 (OP_TRSM_UT) or U^{-1} p1
// (OP_TRSM_U) with the factored b x b leaf p0 (b <= 64); the panel is
// processed in chunks of 64 columns.
#define LDS_TRSM (2 * 64 * 65 * 8 + 64 * 4)
__device__ void d_trsm(const Op& op, char* smem) {
  const PRef L = op.p[0];
  const PRef Y = op.p[1];
  const int b = L.rows;
  const int c = pcols(Y);
  const int type = op.type;
  double (*l)[65] = reinterpret_cast<double (*)[65]>(smem);
  double (*y)[65] = reinterpret_cast<double (*)[65]>(smem + 64 * 65 * 8);
  int* pv = reinterpret_cast<int*>(smem + 2 * 64 * 65 * 8);
  const int tid = threadIdx.x;
  const double* g = reinterpret_cast<const double*>(L.ptr);
  for (int e = tid; e < b * b; e += NT) {
    int i = e % b, j = e / b;
    l[i][j] = g[i + (size_t)j * L.ld];
  }
  if (type == OP_TRSM_L) {
    const int32_t* piv = reinterpret_cast<const int32_t*>(op.p[2].ptr);
    for (int i = tid; i < b; i += NT) pv[i] = piv[i];
  }
  __syncthreads();
  for (int c0 = 0; c0 < c; c0 += 64) {
    const int w = min(64, c - c0);
    for (int e = tid; e < b * w; e += NT) {
      int i = e % b, j = e / b;
      y[i][j] = pget(Y, i, c0 + j);
    }
    __syncthreads();
    if (type == OP_TRSM_L) {
      if (tid < w) {
        for (int k = 0; k < b; ++k) {
          int p = pv[k];
          if (p != k) {
            double t = y[k][tid];
            y[k][tid] = y[p][tid];
            y[p][tid] = t;
          }
        }
      }
      __syncthreads();
      for (int k = 0; k < b - 1; ++k) {
        const int r = b - k - 1;
        for (int e = tid; e < r * w; e += NT) {
          int i = k + 1 + e % r, j = e / r;
          y[i][j] -= l[i][k] * y[k][j];
        }
        __syncthreads();
      }
    } else if (type == OP_TRSM_UT) {
      for (int k = 0; k < b; ++k) {
        if (tid < w) y[k][tid] = y[k][tid] / l[k][k];
        __syncthreads();
        const int r = b - k - 1;
        for (int e = tid; e < r * w; e += NT) {
          int i = k + 1 + e % r, j = e / r;
          y[i][j] -= l[k][i] * y[k][j];
        }
        __syncthreads();
      }
    } else {
      for (int k = b - 1; k >= 0; --k) {
        if (tid < w) y[k][tid] = y[k][tid] / l[k][k];
        __syncthreads();
        for (int e = tid; e < k * w; e += NT) {
          int i = e % k, j = e / k;
          y[i][j] -= l[i][k] * y[k][j];
        }
        __syncthreads();
      }
    }
    for (int e = tid; e < b * w; e += NT) {
      int i = e % b, j = e / b;
      pset(Y, i, c0 + j, y[i][j]);
    }
    __syncthreads();
  }
  const double es = Y.dt == DT_F64 ? 8.0 : 4.0;
  put_cost(op, (double)b * b * c, 8.0 * b * b / 2 + 2.0 * es * b * c);
}

// ---------------------------------------------------------------- panel products
// p3 += d0 * op(M) p2.  Dense M: tiles of 64 x 64 outputs with 32-deep LDS
// slabs.  Low-rank M = A B^T: T = B^T X (k x c) in LDS, then Y += d0 A T.
#define LDS_PGEMM (64 * 33 * 8 + 32 * 65 * 8 + 64 * 65 * 8)
__device__ void d_pgemm(const Op& op, char* smem) {
  const PRef X = op.p[2];
  const PRef Y = op.p[3];
  const double sg = op.d0;
  const int tid = threadIdx.x;
  const int c = pcols(Y) < pcols(X) ? pcols(Y) : pcols(X);
  const int m = Y.rows;
  double (*sa)[33] = reinterpret_cast<double (*)[33]>(smem);
  double (*sb)[65] = reinterpret_cast<double (*)[65]>(smem + 64 * 33 * 8);
  double (*st)[65] = reinterpret_cast<double (*)[65]>(smem + 64 * 33 * 8 + 32 * 65 * 8);
  const int ti = tid % 16, tj = tid / 16;   // 16 x 16 threads, 4 x 4 outputs each
  const double esx = X.dt == DT_F64 ? 8.0 : 4.0;
  const double esy = Y.dt == DT_F64 ? 8.0 : 4.0;
  if (op.i0 == 0) {
    PRef M = op.p[0];
    const bool tr = op.i1 != 0;
    const int r = X.rows;   // inner dimension
    for (int c0 = 0; c0 < c; c0 += 64) {
      const int w = min(64, c - c0);
      for (int r0 = 0; r0 < m; r0 += 64) {
        const int h = min(64, m - r0);
        double acc[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
        for (int k0 = 0; k0 < r; k0 += 32) {
          const int d = min(32, r - k0);
          for (int e = tid; e < 64 * 32; e += NT) {
            int i = e % 64, kk = e / 64;
            double v = 0.0;
            if (i < h && kk < d) v = tr ? pget(M, k0 + kk, r0 + i) : pget(M, r0 + i, k0 + kk);
            sa[i][kk] = v;
          }
          for (int e = tid; e < 32 * 64; e += NT) {
            int kk = e % 32, j = e / 32;
            sb[kk][j] = (kk < d && j < w) ? pget(X, k0 + kk, c0 + j) : 0.0;
          }
          __syncthreads();
          for (int kk = 0; kk < d; ++kk) {
            double av[4], bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) av[u] = sa[ti + 16 * u][kk];
#pragma unroll
            for (int v = 0; v < 4; ++v) bv[v] = sb[kk][tj + 16 * v];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
              for (int v = 0; v < 4; ++v) acc[u][v] += av[u] * bv[v];
          }
          __syncthreads();
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            int i = ti + 16 * u, j = tj + 16 * v;
            if (i < h && j < w) pset(Y, r0 + i, c0 + j, pget(Y, r0 + i, c0 + j) + sg * acc[u][v]);
          }
      }
    }
    put_cost(op, 2.0 * m * r * c, 8.0 * m * r + esx * r * c + 2.0 * esy * m * c);
    return;
  }
  // low-rank M: (A, B) = (U, V) or (V, U) when transposed
  const PRef U = op.p[0], V = op.p[1];
  const bool tr = op.i1 != 0;
  const PRef A = tr ? V : U;
  const PRef B = tr ? U : V;
  const int k = pcols(U);
  const int r = X.rows;
  const double esm = U.dt == DT_F64 ? 8.0 : 4.0;
  for (int c0 = 0; c0 < c; c0 += 64) {
    const int w = min(64, c - c0);
    // T = B^T X  (k x w), k <= 64
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
    for (int k0 = 0; k0 < r; k0 += 32) {
      const int d = min(32, r - k0);
      for (int e = tid; e < 64 * 32; e += NT) {
        int i = e % 64, kk = e / 64;   // i: rank index, kk: row of B
        sa[i][kk] = (i < k && kk < d) ? pget(B, k0 + kk, i) : 0.0;
      }
      for (int e = tid; e < 32 * 64; e += NT) {
        int kk = e % 32, j = e / 32;
        sb[kk][j] = (kk < d && j < w) ? pget(X, k0 + kk, c0 + j) : 0.0;
      }
      __syncthreads();
      for (int kk = 0; kk < d; ++kk) {
        double av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) av[u] = sa[ti + 16 * u][kk];
#pragma unroll
        for (int v = 0; v < 4; ++v) bv[v] = sb[kk][tj + 16 * v];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] += av[u] * bv[v];
      }
      __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) st[ti + 16 * u][tj + 16 * v] = acc[u][v];
    __syncthreads();
    // Y += sg * A T
    for (int r0 = 0; r0 < m; r0 += 64) {
      const int h = min(64, m - r0);
      for (int e = tid; e < 64 * 32; e += NT) {
        int i = e % 64, kk = e / 64;
        sa[i][kk] = (i < h && kk < k && kk < 32) ? pget(A, r0 + i, kk) : 0.0;
      }
      __syncthreads();
      double o[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) o[u][v] = 0.0;
      const int kk_end = min(k, 32);
      for (int kk = 0; kk < kk_end; ++kk) {
        double av[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) av[u] = sa[ti + 16 * u][kk];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) o[u][v] += av[u] * st[kk][tj + 16 * v];
      }
      __syncthreads();
      if (k > 32) {
        for (int e = tid; e < 64 * 32; e += NT) {
          int i = e % 64, kk = e / 64;
          sa[i][kk] = (i < h && 32 + kk < k) ? pget(A, r0 + i, 32 + kk) : 0.0;
        }
        __syncthreads();
        for (int kk = 0; kk < k - 32; ++kk) {
          double av[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) av[u] = sa[ti + 16 * u][kk];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) o[u][v] += av[u] * st[32 + kk][tj + 16 * v];
        }
        __syncthreads();
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          int i = ti + 16 * u, j = tj + 16 * v;
          if (i < h && j < w) pset(Y, r0 + i, c0 + j, pget(Y, r0 + i, c0 + j) + sg * o[u][v]);
        }
    }
    __syncthreads();
  }
  put_cost(op, 2.0 * (double)k * c * (r + m),
           esm * (double)k * (r + m) + esx * r * c + 2.0 * esy * m * c);
}

// ---------------------------------------------------------------- dense update
// p0 (FP64 dense, m x n) -= p1 p2^T
#define LDS_ADDD (64 * 33 * 8 + 32 * 65 * 8)
__device__ void d_addd(const Op& op, char* smem) {
  const PRef C = op.p[0], X = op.p[1], Y = op.p[2];
  const int m = C.rows, n = C.cols;
  const int k = pcols(X);
  double (*sa)[33] = reinterpret_cast<double (*)[33]>(smem);
  double (*sb)[65] = reinterpret_cast<double (*)[65]>(smem + 64 * 33 * 8);
  const int tid = threadIdx.x;
  const int ti = tid % 16, tj = tid / 16;
  double* g = reinterpret_cast<double*>(C.ptr);
  for (int c0 = 0; c0 < n; c0 += 64) {
    const int w = min(64, n - c0);
    for (int r0 = 0; r0 < m; r0 += 64) {
      const int h = min(64, m - r0);
      double acc[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
      for (int k0 = 0; k0 < k; k0 += 32) {
        const int d = min(32, k - k0);
        for (int e = tid; e < 64 * 32; e += NT) {
          int i = e % 64, kk = e / 64;
          sa[i][kk] = (i < h && kk < d) ? pget(X, r0 + i, k0 + kk) : 0.0;
        }
        for (int e = tid; e < 32 * 64; e += NT) {
          int kk = e % 32, j = e / 32;
          sb[kk][j] = (kk < d && j < w) ? pget(Y, c0 + j, k0 + kk) : 0.0;
        }
        __syncthreads();
        for (int kk = 0; kk < d; ++kk) {
          double av[4], bv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) av[u] = sa[ti + 16 * u][kk];
#pragma unroll
          for (int v = 0; v < 4; ++v) bv[v] = sb[kk][tj + 16 * v];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] += av[u] * bv[v];
        }
        __syncthreads();
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          int i = ti + 16 * u, j = tj + 16 * v;
          if (i < h && j < w) g[(r0 + i) + (size_t)(c0 + j) * C.ld] -= acc[u][v];
        }
    }
  }
  const double es = X.dt == DT_F64 ? 8.0 : 4.0;
  put_cost(op, 2.0 * m * n * k, 16.0 * m * n + es * (double)k * (m + n));
}

// ---------------------------------------------------------------- zero
__device__ void d_zero(const Op& op) {
  const PRef Z = op.p[0];
  const int tot = Z.rows * Z.cols;
  for (int e = threadIdx.x; e < tot; e += NT) {
    int i = e % Z.rows, j = e / Z.rows;
    pset(Z, i, j, 0.0);
  }
  put_cost(op, 0.0, (Z.dt == DT_F64 ? 8.0 : 4.0) * tot);
}

// ---------------------------------------------------------------- truncation
// C = U V^T (rank kc) minus a list of low-rank terms X_t Y_t^T (X_t placed at
// row xo_t of C, Y_t at row yo_t, zero elsewhere).  The terms are taken in
// passes whose stacked width K = kc + sum k_t stays <= 64 (live ranks read at
// run time); every pass replaces C by the best approximation of
// [U, -X_a, ..., -X_b] [V, Y_a, ..., Y_b]^T:
//   1. Gram matrices Gx = Xs^T Xs, Gy = Ys^T Ys in FP64 (rows streamed in
//      chunks of 64, only the K live columns, 4x4 blocks per thread over
//      row groups);
//   2. column balancing so that |x_j| = |y_j|;
//   3. pivoted Cholesky Gx = Pi_x R^T R Pi_x^T, Gy = Pi_y S^T S Pi_y^T,
//      stopping at pivots below 1e-14 of the largest diagonal;
//   4. M = R S^T and its one-sided Jacobi SVD M = W Sig Z^T;
//   5. rank choice (fixed, or the smallest k with discarded Frobenius norm
//      <= eps |Sig|, capped);
//   6. Tx = D Pi_x R11^{-1} W_k Sig_k, Ty = D^{-1} Pi_y S11^{-1} Z_k;
//   7. U := Xs Tx, V := Ys Ty streamed in place (each row chunk is read
//      before it is written).
#define KM 64
#define TMAX 16
struct TruncShared {
  double gx[KM][KM + 1];    // Gx -> R -> (after step 6) Ty
  double gy[KM][KM + 1];    // Gy -> S
  double m[KM][KM + 1];     // row chunks / M -> W Sig / row chunks
  double z[KM][KM + 1];     // Gram partials / Z
  double tt[KM][33];        // Tx
  double dsc[KM];
  double sig[KM];
  Term tm[TMAX];            // terms of the current pass
  int px[KM], py[KM], posx[KM], posy[KM], ord[KM];
  int8_t colt[KM], colj[KM];   // stacked column -> (term, column in term)
  int rx, ry, k, rot, capped, sp, K, kc, tb, te;
  double sdmax, mnorm;
};

// element (i, j) of the stacked panel of one side (0: [U, -X..], 1: [V, Y..])
__device__ __forceinline__ double stk(const TruncShared& sh, const PRef& F, int side, int i,
                                      int j) {
  if (j < sh.kc) return pget(F, i, j);
  const Term& t = sh.tm[sh.colt[j]];
  const int ii = i - (side ? t.yo : t.xo);
  const PRef& T = side ? t.Y : t.X;
  if (ii < 0 || ii >= T.rows) return 0.0;
  const double v = pget(T, ii, sh.colj[j]);
  return side ? v : -v;
}

__device__ __forceinline__ void trunc_load_chunk(TruncShared& sh, const PRef& F, int side, int r0,
                                                 int h, int K) {
  for (int e = threadIdx.x; e < 64 * K; e += NT) {
    int i = e % 64, j = e / 64;
    sh.m[i][j] = i < h ? stk(sh, F, side, r0 + i, j) : 0.0;
  }
}

// G (K x K) = S^T S of the stacked panel of one side
__device__ void trunc_gram(TruncShared& sh, double (*G)[KM + 1], const PRef& F, int side,
                           int rows, int K) {
  const int tid = threadIdx.x;
  const int B = (K + 3) / 4;
  const int BB = B * B;
  const int NG = BB > 0 ? min(NT / BB, 16) : 1;
  const int grp = BB > 0 ? tid / BB : 0, blk = BB > 0 ? tid % BB : 0;
  const bool act = BB > 0 && grp < NG;
  const int bi = act ? blk / B : 0, bj = act ? blk % B : 0;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int r0 = 0; r0 < rows; r0 += 64) {
    const int h = min(64, rows - r0);
    trunc_load_chunk(sh, F, side, r0, h, K);
    __syncthreads();
    if (act) {
      for (int i = grp; i < h; i += NG) {
        double av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          int a = 4 * bi + u, b = 4 * bj + u;
          av[u] = a < K ? sh.m[i][a] : 0.0;
          bv[u] = b < K ? sh.m[i][b] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] += av[u] * bv[v];
      }
    }
    __syncthreads();
  }
  double* part = &sh.z[0][0];
  if (act) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) part[(size_t)(grp * BB + blk) * 16 + u * 4 + v] = acc[u][v];
  }
  __syncthreads();
  for (int e = tid; e < K * K; e += NT) {
    int a = e % K, b = e / K;
    int q = ((a / 4) * B + (b / 4)) * 16 + (a % 4) * 4 + (b % 4);
    double s = 0.0;
    for (int g = 0; g < NG; ++g) s += part[(size_t)g * BB * 16 + q];
    G[a][b] = s;
  }
  __syncthreads();
}

// In-place pivoted Cholesky of G (K x K).  On exit rows piv[0..r) of G hold
// the rows of R in stacked-column order (entries of columns eliminated
// before a row's own pivot are zero), pos[c] is the pivot position of
// column c, and r the numerical rank.
__device__ void trunc_pchol(TruncShared& sh, double (*G)[KM + 1], int* piv, int* pos, int K,
                            int* r_out) {
  const int tid = threadIdx.x;
  for (int j = tid; j < KM; j += NT) piv[j] = j;
  __syncthreads();
  double dmax0 = 0.0;
  for (int j = 0; j < K; ++j) dmax0 = fmax(dmax0, G[j][j]);
  int r = 0;
  for (int step = 0; step < K; ++step) {
    if (tid < 64) {
      const int q = tid;
      double v = (q >= step && q < K) ? G[piv[q]][piv[q]] : -1.0;
      int ix = q;
      for (int o = 32; o > 0; o >>= 1) {
        double v2 = __shfl_xor(v, o);
        int i2 = __shfl_xor(ix, o);
        if (v2 > v || (v2 == v && i2 < ix)) { v = v2; ix = i2; }
      }
      if (tid == 0) {
        int t = piv[step];
        piv[step] = piv[ix];
        piv[ix] = t;
        sh.sdmax = v;
        sh.sp = piv[step];
      }
    }
    __syncthreads();
    if (!(sh.sdmax > 1e-14 * dmax0) || !(dmax0 > 0.0)) break;
    const int p = sh.sp;
    const double rp = sqrt(sh.sdmax);
    for (int q = step + tid; q < K; q += NT) {
      int c = piv[q];
      G[p][c] = (q == step) ? rp : G[p][c] / rp;
    }
    __syncthreads();
    const int rem = K - step - 1;
    for (int e = tid; e < rem * rem; e += NT) {
      int a = piv[step + 1 + e % rem], b = piv[step + 1 + e / rem];
      G[a][b] -= G[p][a] * G[p][b];
    }
    __syncthreads();
    ++r;
  }
  for (int q = tid; q < K; q += NT) pos[piv[q]] = q;
  __syncthreads();
  for (int e = tid; e < r * K; e += NT) {
    int i = e % r, c = e / r;
    if (pos[c] < i) G[piv[i]][c] = 0.0;
  }
  if (tid == 0) *r_out = r;
  __syncthreads();
}

// Column-oriented back substitution: out[c2][c] (stacked column c2, kept
// singular vector c) = D^{+-1} Pi R11^{-1} src[:, ord[c]].
__device__ void trunc_backsub(TruncShared& sh, double (*G)[KM + 1], const int* pv, int r,
                              double (*src)[KM + 1], double (*out)[33], int K, int k,
                              bool scale_mul) {
  const int tid = threadIdx.x;
  for (int e = tid; e < KM * 33; e += NT) out[e % KM][e / KM] = 0.0;
  __syncthreads();
  for (int e = tid; e < r * k; e += NT) {
    int i = e % r, c = e / r;
    out[pv[i]][c] = src[i][sh.ord[c]];
  }
  __syncthreads();
  for (int i = r - 1; i >= 0; --i) {
    const int pi = pv[i];
    if (tid < k) out[pi][tid] /= G[pi][pi];
    __syncthreads();
    for (int e = tid; e < i * k; e += NT) {
      int j = e % i, c = e / i;
      out[pv[j]][c] -= G[pv[j]][pi] * out[pi][c];
    }
    __syncthreads();
  }
  for (int e = tid; e < K * k; e += NT) {
    int c2 = e % K, c = e / K;
    double dd = sh.dsc[c2];
    out[c2][c] = scale_mul ? out[c2][c] * dd : (dd > 0.0 ? out[c2][c] / dd : 0.0);
  }
  __syncthreads();
}

// rows of F := stacked rows . T  (T: K x k, in place, chunks of 64 rows)
__device__ void trunc_apply(TruncShared& sh, const PRef& F, int side, int rows, int K, int k,
                            double (*T)[33]) {
  const int tid = threadIdx.x;
  const int i = tid % 64, cb = tid / 64;
  for (int r0 = 0; r0 < rows; r0 += 64) {
    const int h = min(64, rows - r0);
    trunc_load_chunk(sh, F, side, r0, h, K);
    __syncthreads();
    if (i < h && cb * 8 < k) {
      const int c0 = cb * 8;
      double o[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) o[v] = 0.0;
      for (int c2 = 0; c2 < K; ++c2) {
        const double a = sh.m[i][c2];
#pragma unroll
        for (int v = 0; v < 8; ++v) o[v] += a * T[c2][c0 + v];
      }
#pragma unroll
      for (int v = 0; v < 8; ++v)
        if (c0 + v < k) pset(F, r0 + i, c0 + v, o[v]);
    }
    __syncthreads();
  }
}

#define LDS_TRUNC (sizeof(TruncShared))
__device__ void d_trunc(const Op& op, char* smem) {
  const PRef U = op.p[0], V = op.p[1];
  const Term* terms = reinterpret_cast<const Term*>(op.p[2].ptr) + op.i0;
  const int nterms = op.i1;
  const int cap = op.i2 & 0xffff, fixed = op.i2 >> 16;
  const double eps = op.d0;
  const int m = U.rows, n = V.rows;
  TruncShared& sh = *reinterpret_cast<TruncShared*>(smem);
  const int tid = threadIdx.x;
  double flops = 0.0, bytes = 0.0;
  const double es = U.dt == DT_F64 ? 8.0 : 4.0;
  int capped_any = 0, Kmax = 0;
  if (tid == 0) sh.te = 0;
  __syncthreads();
  while (sh.te < nterms) {
    // choose this pass's terms and map the stacked columns
    if (tid == 0) {
      const int kc = pcols(U);
      int K = kc, t = sh.te, c = 0;
      const int tb = t;
      while (t < nterms && t - tb < TMAX) {
        const int w = pcols(terms[t].X);
        if (t > tb && K + w > KM) break;
        for (int j = 0; j < w; ++j) {
          sh.colt[K + j] = (int8_t)(t - tb);
          sh.colj[K + j] = (int8_t)j;
        }
        sh.tm[t - tb] = terms[t];
        K += w;
        ++t;
        ++c;
      }
      sh.kc = kc;
      sh.K = K;
      sh.tb = tb;
      sh.te = t;
      sh.capped = 0;
    }
    __syncthreads();
    const int K = sh.K, kc = sh.kc;
    Kmax = max(Kmax, K);
    // 1. Gram matrices
    trunc_gram(sh, sh.gx, U, 0, m, K);
    trunc_gram(sh, sh.gy, V, 1, n, K);
    // 2. balancing
    for (int j = tid; j < K; j += NT) {
      double a = sh.gx[j][j], b = sh.gy[j][j];
      sh.dsc[j] = (a > 0.0 && b > 0.0) ? sqrt(sqrt(b / a)) : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < K * K; e += NT) {
      int a = e % K, b = e / K;
      double da = sh.dsc[a], db = sh.dsc[b];
      sh.gx[a][b] *= da * db;
      sh.gy[a][b] = (da > 0.0 && db > 0.0) ? sh.gy[a][b] / (da * db) : 0.0;
    }
    __syncthreads();
    // 3. pivoted Cholesky of both sides
    trunc_pchol(sh, sh.gx, sh.px, sh.posx, K, &sh.rx);
    trunc_pchol(sh, sh.gy, sh.py, sh.posy, K, &sh.ry);
    const int rx = sh.rx, ry = sh.ry;
    // 4. M = R S^T (rows in pivot order), Z = I
    {
      const int ti = tid % 16, tj = tid / 16;
      double acc[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
      int ra[4], sb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        ra[u] = (ti + 16 * u < rx) ? sh.px[ti + 16 * u] : -1;
        sb[u] = (tj + 16 * u < ry) ? sh.py[tj + 16 * u] : -1;
      }
      for (int c = 0; c < K; ++c) {
        double av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) av[u] = ra[u] >= 0 ? sh.gx[ra[u]][c] : 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) bv[v] = sb[v] >= 0 ? sh.gy[sb[v]][c] : 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] += av[u] * bv[v];
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) sh.m[ti + 16 * u][tj + 16 * v] = acc[u][v];
    }
    for (int e = tid; e < KM * KM; e += NT) {
      int i = e % KM, j = e / KM;
      sh.z[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (tid < 64) {
      double s = 0.0;
      for (int e = tid; e < rx * ry; e += 64) {
        const double v = sh.m[e % rx][e / rx];
        s += v * v;
      }
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
      if (tid == 0) sh.mnorm = s;
    }
    __syncthreads();
    const double ms = sh.mnorm;
    // one-sided Jacobi on the columns of M (rx rows, ry columns)
    const int ncol = ry + (ry & 1);
    const double tiny = 1e-30 * ms;
    if (ncol >= 2 && rx > 0 && ms > 0.0) {
      const int npair = ncol / 2;
      int grp = 64;
      while (grp > 1 && grp * npair > NT) grp >>= 1;   // threads per pair
      const int q = tid / grp, l = tid % grp;
      for (int sweep = 0; sweep < 24; ++sweep) {
        if (tid == 0) sh.rot = 0;
        __syncthreads();
        for (int round = 0; round < ncol - 1; ++round) {
          if (q < npair) {
            int x0 = (q == 0) ? ncol - 1 : (round + q) % (ncol - 1);
            int x1 = (q == 0) ? round % (ncol - 1) : (round + ncol - 1 - q) % (ncol - 1);
            const int a = min(x0, x1), b = max(x0, x1);
            double al = 0, be = 0, ga = 0;
            const bool valid = b < ry;
            if (valid) {
              for (int i = l; i < rx; i += grp) {
                double u = sh.m[i][a], v = sh.m[i][b];
                al += u * u;
                be += v * v;
                ga += u * v;
              }
            }
            for (int o = grp / 2; o > 0; o >>= 1) {
              al += __shfl_xor(al, o);
              be += __shfl_xor(be, o);
              ga += __shfl_xor(ga, o);
            }
            if (valid && al > tiny && be > tiny && fabs(ga) > 1e-15 * sqrt(al * be)) {
              double zeta = (be - al) / (2.0 * ga);
              double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
              double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
              for (int i = l; i < rx; i += grp) {
                double u = sh.m[i][a], v = sh.m[i][b];
                sh.m[i][a] = cs * u - sn * v;
                sh.m[i][b] = sn * u + cs * v;
              }
              for (int i = l; i < ry; i += grp) {
                double u = sh.z[i][a], v = sh.z[i][b];
                sh.z[i][a] = cs * u - sn * v;
                sh.z[i][b] = sn * u + cs * v;
              }
              if (l == 0) sh.rot = 1;
            }
          }
          __syncthreads();
        }
        if (!sh.rot) break;
        __syncthreads();
      }
    }
    // singular values, descending order (stable), rank choice
    const int nr = rx > 0 ? ry : 0;
    for (int j = tid; j < nr; j += NT) {
      double s = 0.0;
      for (int i = 0; i < rx; ++i) s += sh.m[i][j] * sh.m[i][j];
      sh.sig[j] = sqrt(s);
    }
    __syncthreads();
    for (int j = tid; j < nr; j += NT) {
      const double sj = sh.sig[j];
      int c = 0;
      for (int i = 0; i < nr; ++i) {
        const double si = sh.sig[i];
        c += (si > sj || (si == sj && i < j)) ? 1 : 0;
      }
      sh.ord[c] = j;
    }
    __syncthreads();
    if (tid == 0) {
      const int lim = min(nr, rx);
      int k;
      if (fixed > 0) {
        k = min(fixed, lim);
      } else {
        double tot = 0.0;
        for (int j = 0; j < nr; ++j) tot += sh.sig[j] * sh.sig[j];
        const double thr = eps * eps * tot;
        double tail = 0.0;
        k = nr;
        for (int j = nr; j >= 0; --j) {
          if (tail <= thr) k = j;
          else break;
          if (j > 0) tail += sh.sig[sh.ord[j - 1]] * sh.sig[sh.ord[j - 1]];
        }
        k = min(k, lim);
        if (k > cap) {
          k = cap;
          sh.capped = 1;
        }
      }
      sh.k = k;
    }
    __syncthreads();
    const int k = sh.k;
    capped_any |= sh.capped;
    // 6. Tx into tt; Ty into the space of gx (R is no longer needed)
    trunc_backsub(sh, sh.gx, sh.px, rx, sh.m, sh.tt, K, k, true);
    double (*ty)[33] = reinterpret_cast<double (*)[33]>(&sh.gx[0][0]);
    trunc_backsub(sh, sh.gy, sh.py, ry, sh.z, ty, K, k, false);
    // 7. new factors, streamed in place; then the new rank
    trunc_apply(sh, U, 0, m, K, k, sh.tt);
    trunc_apply(sh, V, 1, n, K, k, ty);
    if (tid == 0) *reinterpret_cast<int32_t*>(U.rankp) = k;
    __threadfence_block();
    __syncthreads();
    flops += 2.0 * (m + n) * K * K - 4.0 * K * K * K / 3.0 + 2.0 * K * K * K +
             21.0 * K * K * K + 2.0 * (m + n) * K * k;
    bytes += es * (double)(m + n) * (K + k);
  }
  put_cost(op, flops, bytes, (double)capped_any, (double)sh.k, (double)Kmax);
}

// ---------------------------------------------------------------- matvec
// T_b = V_b^T X[c0:c0+n, :] for every low-rank block b of the matvec copy.
__global__ void __launch_bounds__(NT) k_mv_t(const MvLR* __restrict__ lr, const double* X,
                                             int ldx, int nrhs) {
  const MvLR e = lr[blockIdx.x];
  if (e.k == 0) return;
  const double* V = reinterpret_cast<const double*>(e.V);
  double* T = reinterpret_cast<double*>(e.T);
  __shared__ double sv[32][65];
  __shared__ double sx[32][65];
  const int tid = threadIdx.x;
  const int ti = tid % 16, tj = tid / 16;
  for (int k0 = 0; k0 < e.k; k0 += 64) {
    const int kk = min(64, e.k - k0);
    for (int c0 = 0; c0 < nrhs; c0 += 64) {
      const int w = min(64, nrhs - c0);
      double acc[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
      for (int r0 = 0; r0 < e.n; r0 += 32) {
        const int d = min(32, e.n - r0);
        for (int q = tid; q < 32 * 64; q += NT) {
          int i = q % 32, j = q / 32;
          sv[i][j] = (i < d && j < kk) ? V[(r0 + i) + (size_t)(k0 + j) * e.n] : 0.0;
          sx[i][j] = (i < d && j < w) ? X[(e.c0 + r0 + i) + (size_t)(c0 + j) * ldx] : 0.0;
        }
        __syncthreads();
        for (int i = 0; i < d; ++i) {
          double av[4], bv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) av[u] = sv[i][ti + 16 * u];
#pragma unroll
          for (int v = 0; v < 4; ++v) bv[v] = sx[i][tj + 16 * v];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] += av[u] * bv[v];
        }
        __syncthreads();
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          int a = ti + 16 * u, b = tj + 16 * v;
          if (a < kk && b < w) T[(k0 + a) + (size_t)(c0 + b) * e.kcap] = acc[u][v];
        }
    }
  }
}

// y[rows of leaf] = beta * b + alpha * sum over the leaf row's blocks (F X or
// U T): (0, 1) gives y = A X, (1, -1) the residual b - A X.
__global__ void __launch_bounds__(NT) k_mv_rows(const MvRow* __restrict__ rows,
                                                const MvTerm* __restrict__ terms,
                                                const double* X, int ldx, const double* B,
                                                double beta, double alpha, double* Yo,
                                                int nrhs) {
  const MvRow r = rows[blockIdx.x];
  const int tid = threadIdx.x;
  for (int c0 = 0; c0 < nrhs; c0 += 4) {
    // each thread: row i = tid % 64, column c0 + tid / 64
    const int i = tid % 64, j = c0 + tid / 64;
    double acc = 0.0;
    const bool act = i < r.rows && j < nrhs;
    for (int q = 0; q < r.nt; ++q) {
      const MvTerm t = terms[r.t0 + q];
      const double* A = reinterpret_cast<const double*>(t.A);
      if (!act) continue;
      if (t.T == 0) {
        const double* x = X + (size_t)j * ldx + t.c0;
        for (int c = 0; c < t.ncol; ++c) acc += A[(t.roff + i) + (size_t)c * t.lda] * x[c];
      } else {
        const double* T = reinterpret_cast<const double*>(t.T) + (size_t)j * t.c0;
        for (int c = 0; c < t.ncol; ++c) acc += A[(t.roff + i) + (size_t)c * t.lda] * T[c];
      }
    }
    if (act) {
      size_t o = (size_t)(r.r0 + i) + (size_t)j * ldx;
      Yo[o] = beta * (B ? B[o] : 0.0) + alpha * acc;
    }
  }
}

// ---------------------------------------------------------------- vectors
__global__ void k_gather(const double* b, int64_t ldb, double* Y, int ldy, const int64_t* perm,
                         int n, int nrhs) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * nrhs) return;
  int p = (int)(e % n), j = (int)(e / n);
  Y[p + (size_t)j * ldy] = b[perm[p] + (size_t)j * ldb];
}

__global__ void k_scatter(const double* Y, int ldy, double* x, int64_t ldx, const int64_t* perm,
                          int n, int nrhs) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * nrhs) return;
  int p = (int)(e % n), j = (int)(e / n);
  x[perm[p] + (size_t)j * ldx] = Y[p + (size_t)j * ldy];
}

__global__ void k_axpy(double* X, const double* D, int ld, int n, int nrhs, double a) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * nrhs) return;
  int p = (int)(e % n), j = (int)(e / n);
  X[p + (size_t)j * ld] = (a == 0.0 ? 0.0 : X[p + (size_t)j * ld]) + D[p + (size_t)j * ld];
}

// per column j: out[3j] = max|R_j|, out[3j+1] = max|X_j|, out[3j+2] = max|B_j|
__global__ void __launch_bounds__(NT) k_colmax(const double* R, const double* X, const double* B,
                                               int ld, int n, double* out) {
  const int j = blockIdx.x;
  const int tid = threadIdx.x;
  __shared__ double red[3][NT];
  double a = 0, b = 0, c = 0;
  for (int i = tid; i < n; i += NT) {
    size_t o = (size_t)i + (size_t)j * ld;
    a = fmax(a, fabs(R[o]));
    b = fmax(b, fabs(X[o]));
    c = fmax(c, fabs(B[o]));
  }
  red[0][tid] = a;
  red[1][tid] = b;
  red[2][tid] = c;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s)
      for (int q = 0; q < 3; ++q) red[q][tid] = fmax(red[q][tid], red[q][tid + s]);
    __syncthreads();
  }
  if (tid < 3) out[3 * j + tid] = red[tid][0];
}

__global__ void k_set_int(int32_t* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// ---------------------------------------------------------------- launchers
// One workgroup per descriptor; the descriptors of a launch may mix op
// types (one launch per wave of the schedule).  Each op type carves its
// tiles out of the same dynamic LDS buffer, so a launch requests the
// largest footprint among the types it contains.
__device__ __forceinline__ void run_op(const Op& op, char* smem) {
  start_tick(op);
  switch (op.type) {
    case OP_GETRF: d_getrf(op, smem); break;
    case OP_TRSM_L:
    case OP_TRSM_UT:
    case OP_TRSM_U: d_trsm(op, smem); break;
    case OP_PGEMM: d_pgemm(op, smem); break;
    case OP_TRUNC: d_trunc(op, smem); break;
    case OP_ADDD: d_addd(op, smem); break;
    case OP_ZERO: d_zero(op); break;
    default: break;
  }
}

__global__ void __launch_bounds__(NT) k_wave(const Op* __restrict__ ops) {
  extern __shared__ __align__(16) char smem[];
  run_op(ops[blockIdx.x], smem);
}

// ---------------------------------------------------------------- dataflow
// Persistent executor of the whole factor schedule: the device analogue of
// running nested tasks with weak dependencies and early release (Sec. 4.3)
// -- an op starts as soon as its own predecessors have finished, across
// recursion levels, instead of waiting for a whole wave.
//   ctrl[0]: next queue slot to take, ctrl[1]: next slot to fill,
//   ctrl[2]: error flag (a wait exceeded the time limit).
// Every op is pushed exactly once (when its last predecessor finishes), so
// the queue has one slot per op; a workgroup that takes a slot >= n exits.
// Waits are bounded by `timeout` ticks of the constant-rate wall clock, after
// which the error flag is raised and every waiting workgroup exits.
__global__ void k_df_reset(int* indeg, const int* indeg0, int* queue, const int* ready0,
                           int nready, int n, int* ctrl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    indeg[i] = indeg0[i];
    queue[i] = i < nready ? ready0[i] : -1;
  }
  if (i == 0) {
    ctrl[0] = 0;
    ctrl[1] = nready;
    ctrl[2] = 0;
  }
}

__global__ void __launch_bounds__(NT) k_dataflow(const Op* __restrict__ ops,
                                                 const int* __restrict__ succ_off,
                                                 const int* __restrict__ succ, int* indeg,
                                                 int* queue, int* ctrl, int n,
                                                 long long timeout) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_op;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) {
      int v = -1;
      const int s = __hip_atomic_fetch_add(&ctrl[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (s < n) {
        const long long t0 = (long long)wall_clock64();
        for (;;) {
          v = __hip_atomic_load(&queue[s], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
          if (v >= 0) break;
          if (__hip_atomic_load(&ctrl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
          if ((long long)wall_clock64() - t0 > timeout) {
            __hip_atomic_store(&ctrl[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
      s_op = v;
    }
    __syncthreads();
    const int idx = s_op;
    if (idx < 0) break;
    run_op(ops[idx], smem);
    __syncthreads();
    if (tid == 0) {
      __threadfence();
      for (int e = succ_off[idx]; e < succ_off[idx + 1]; ++e) {
        const int t = succ[e];
        if (__hip_atomic_fetch_add(&indeg[t], -1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == 1) {
          const int slot =
              __hip_atomic_fetch_add(&ctrl[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (slot < n)
            __hip_atomic_store(&queue[slot], t, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
          else
            __hip_atomic_store(&ctrl[2], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    __syncthreads();
  }
}

static size_t lds_bytes(int type) {
  switch (type) {
    case OP_GETRF: return LDS_GETRF;
    case OP_TRSM_L:
    case OP_TRSM_UT:
    case OP_TRSM_U: return LDS_TRSM;
    case OP_PGEMM: return LDS_PGEMM;
    case OP_TRUNC: return LDS_TRUNC;
    case OP_ADDD: return LDS_ADDD;
    default: return 0;
  }
}

static hipError_t launch_wave(const Op* ops, int count, size_t lds, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_wave),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)LDS_TRUNC);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k_wave, dim3(count), dim3(NT), lds, s, ops);
  return hipGetLastError();
}

static hipError_t launch_ops(int type, const Op* ops, int count, hipStream_t s) {
  if (type < 0 || type >= OP_NTYPES) return hipErrorInvalidValue;
  return launch_wave(ops, count, lds_bytes(type), s);
}

}  // namespace hlu

extern "C" size_t hlu_lds_bytes(int type) { return hlu::lds_bytes(type); }

// Dataflow execution of a schedule: reset kernel + persistent kernel with
// `workers` workgroups (LDS of the largest op type).
static hipError_t df_attr() {
  static bool done = false;
  if (done) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&hlu::k_dataflow),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)sizeof(hlu::TruncShared));
  if (e == hipSuccess) done = true;
  return e;
}

extern "C" hipError_t hlu_launch_dataflow(const void* ops, const int* succ_off, const int* succ,
                                          const int* indeg0, int* indeg, int* queue,
                                          const int* ready0, int nready, int* ctrl, int n,
                                          int workers, long long timeout, hipStream_t s) {
  hipError_t e = df_attr();
  if (e != hipSuccess) return e;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(hlu::k_df_reset, dim3((n + 255) / 256), dim3(256), 0, s, indeg, indeg0,
                     queue, ready0, nready, n, ctrl);
  hipLaunchKernelGGL(hlu::k_dataflow, dim3(workers), dim3(NT), sizeof(hlu::TruncShared), s,
                     reinterpret_cast<const hlu::Op*>(ops), succ_off, succ, indeg, queue, ctrl, n,
                     timeout);
  return hipGetLastError();
}

extern "C" hipError_t hlu_build_df_graph(const void* ops_p, const int* succ_off, const int* succ,
                                         const int* indeg0, int* indeg, int* queue,
                                         const int* ready0, int nready, int* ctrl, int n,
                                         int workers, long long timeout, int32_t* status,
                                         hipGraphExec_t* out) {
  *out = nullptr;
  hipError_t e = df_attr();
  if (e != hipSuccess) return e;
  hipGraph_t g;
  e = hipGraphCreate(&g, 0);
  if (e != hipSuccess) return e;
  hipGraphNode_t n0, n1, n2;
  {
    int zero = 0;
    void* args[] = {&status, &zero};
    hipKernelNodeParams p = {};
    p.func = reinterpret_cast<void*>(&hlu::k_set_int);
    p.gridDim = dim3(1);
    p.blockDim = dim3(64);
    p.kernelParams = args;
    e = hipGraphAddKernelNode(&n0, g, nullptr, 0, &p);
  }
  if (e == hipSuccess) {
    void* args[] = {&indeg, &indeg0, &queue, &ready0, &nready, &n, &ctrl};
    hipKernelNodeParams p = {};
    p.func = reinterpret_cast<void*>(&hlu::k_df_reset);
    p.gridDim = dim3((n + 255) / 256);
    p.blockDim = dim3(256);
    p.kernelParams = args;
    e = hipGraphAddKernelNode(&n1, g, &n0, 1, &p);
  }
  if (e == hipSuccess) {
    const hlu::Op* ops = reinterpret_cast<const hlu::Op*>(ops_p);
    void* args[] = {&ops, &succ_off, &succ, &indeg, &queue, &ctrl, &n, &timeout};
    hipKernelNodeParams p = {};
    p.func = reinterpret_cast<void*>(&hlu::k_dataflow);
    p.gridDim = dim3(workers);
    p.blockDim = dim3(NT);
    p.sharedMemBytes = (unsigned)sizeof(hlu::TruncShared);
    p.kernelParams = args;
    e = hipGraphAddKernelNode(&n2, g, &n1, 1, &p);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  return e;
}

// A graph that replays a schedule: a kernel node resetting the status word
// (when given), then one k_wave node per wave, each depending on the
// previous one.  Built explicitly (no stream capture).
extern "C" hipError_t hlu_build_wave_graph(const void* ops_base, const int* starts,
                                           const int* counts, const size_t* lds, int nwaves,
                                           int32_t* status, hipGraphExec_t* out) {
  *out = nullptr;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&hlu::k_wave),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)sizeof(hlu::TruncShared));
  if (e != hipSuccess) return e;
  hipGraph_t g;
  e = hipGraphCreate(&g, 0);
  if (e != hipSuccess) return e;
  hipGraphNode_t prev = nullptr;
  if (status) {
    hipKernelNodeParams p = {};
    int zero = 0;
    void* args[] = {&status, &zero};
    p.func = reinterpret_cast<void*>(&hlu::k_set_int);
    p.gridDim = dim3(1);
    p.blockDim = dim3(64);
    p.sharedMemBytes = 0;
    p.kernelParams = args;
    p.extra = nullptr;
    e = hipGraphAddKernelNode(&prev, g, nullptr, 0, &p);
    if (e != hipSuccess) { hipGraphDestroy(g); return e; }
  }
  for (int w = 0; w < nwaves && e == hipSuccess; ++w) {
    if (counts[w] <= 0) continue;
    const hlu::Op* ops = reinterpret_cast<const hlu::Op*>(ops_base) + starts[w];
    hipKernelNodeParams p = {};
    void* args[] = {&ops};
    p.func = reinterpret_cast<void*>(&hlu::k_wave);
    p.gridDim = dim3(counts[w]);
    p.blockDim = dim3(NT);
    p.sharedMemBytes = (unsigned)lds[w];
    p.kernelParams = args;
    p.extra = nullptr;
    hipGraphNode_t node;
    e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &p);
    prev = node;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  return e;
}

extern "C" hipError_t hlu_launch_wave(const void* ops, int count, size_t lds, hipStream_t s) {
  return hlu::launch_wave(reinterpret_cast<const hlu::Op*>(ops), count, lds, s);
}

extern "C" hipError_t hlu_launch_ops(int type, const void* ops, int count, hipStream_t s) {
  return hlu::launch_ops(type, reinterpret_cast<const hlu::Op*>(ops), count, s);
}

extern "C" hipError_t hlu_launch_mv(const void* lr, int nlr, const void* rows, int nrows,
                                    const void* terms, const double* X, int ldx, const double* B,
                                    double beta, double alpha, double* Y, int nrhs,
                                    hipStream_t s) {
  if (nlr > 0)
    hipLaunchKernelGGL(hlu::k_mv_t, dim3(nlr), dim3(NT), 0, s,
                       reinterpret_cast<const hlu::MvLR*>(lr), X, ldx, nrhs);
  if (nrows > 0)
    hipLaunchKernelGGL(hlu::k_mv_rows, dim3(nrows), dim3(NT), 0, s,
                       reinterpret_cast<const hlu::MvRow*>(rows),
                       reinterpret_cast<const hlu::MvTerm*>(terms), X, ldx, B, beta, alpha, Y,
                       nrhs);
  return hipGetLastError();
}

extern "C" hipError_t hlu_launch_vec(int what, const double* a, int64_t lda, double* y, int ldy,
                                     const int64_t* perm, int n, int nrhs, hipStream_t s) {
  int64_t tot = (int64_t)n * nrhs;
  dim3 g((unsigned)((tot + 255) / 256)), b(256);
  if (tot == 0) return hipSuccess;
  if (what == 0) hipLaunchKernelGGL(hlu::k_gather, g, b, 0, s, a, lda, y, ldy, perm, n, nrhs);
  else if (what == 1)
    hipLaunchKernelGGL(hlu::k_scatter, g, b, 0, s, a, ldy, y, lda, perm, n, nrhs);
  else if (what == 2) hipLaunchKernelGGL(hlu::k_axpy, g, b, 0, s, y, a, ldy, n, nrhs, 1.0);
  else if (what == 3) hipLaunchKernelGGL(hlu::k_axpy, g, b, 0, s, y, a, ldy, n, nrhs, 0.0);
  return hipGetLastError();
}

extern "C" hipError_t hlu_launch_colmax(const double* R, const double* X, const double* B, int ld,
                                        int n, int nrhs, double* out, hipStream_t s) {
  hipLaunchKernelGGL(hlu::k_colmax, dim3(nrhs), dim3(NT), 0, s, R, X, B, ld, n, out);
  return hipGetLastError();
}

extern "C" hipError_t hlu_launch_set_int(int32_t* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(hlu::k_set_int, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}
