// HIP kernels of the H-LU library (gfx950).
//
// Every kernel of the factorisation schedule processes one descriptor per
// workgroup (256 threads = four 64-wide wavefronts); a launch covers one
// batch (all descriptors of one type in one wave of the schedule).  Small
// tiles are staged through LDS; low-rank panels are streamed in row chunks.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "ops.h"

namespace hlu {

#define NT 256

// The dynamic LDS of every kernel here.  The op bodies take their tiles from
// this array rather than from a pointer argument, so their accesses stay LDS
// accesses even when a body is compiled out of line.
extern __shared__ __align__(16) char hlu_lds[];

// Device data reached through descriptor fields (64-bit addresses) is
// accessed through global-address-space pointers: generic (flat) accesses
// also count against the LDS wait counter, so every LDS access of an op
// would wait for the op's outstanding global loads and stores.
#define HLU_G __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ HLU_G T* gptr(uint64_t a) {
  return (HLU_G T*)a;
}

// live column count: ranks change while a schedule runs, so they are read
// with a device-scope atomic load (never through a cached scalar load)
__device__ __forceinline__ int pcols(const PRef& r) {
  return r.rankp ? __hip_atomic_load(gptr<int32_t>(r.rankp), __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT)
                 : r.cols;
}

// Batched panel access.  Element (i, j) of a stored panel sits at
// i * si + j * sj elements from its start (a transposed panel swaps the two
// strides; `tr` transposes the view once more).  A batch of loads takes one
// uniform branch on the element type around all of its loads, and every
// index must lie inside the panel: callers clamp the indices of lanes they
// do not need and zero those values after the batch.  (Selecting zero per
// element instead would write a register that a load is still filling, and
// the compiler then waits for each load before issuing the next.)  An
// identity panel (element (i, j) is one iff j == i + diag, read only) is
// evaluated instead of loaded.
struct GView {
  uint64_t ptr;
  int64_t si, sj;
  bool f64, ident, tr;
  int diag;
};
__device__ __forceinline__ GView gview(const PRef& r, bool tr = false) {
  const bool t = (r.trans != 0) != tr;
  GView g;
  g.ptr = r.ptr;
  g.si = t ? (int64_t)r.ld : 1;
  g.sj = t ? 1 : (int64_t)r.ld;
  g.f64 = r.dt == DT_F64;
  g.ident = r.kind == PK_IDENT;
  g.tr = tr;
  g.diag = r.ld;
  return g;
}
template <int N>
__device__ __forceinline__ void gload(const GView& g, const int (&i)[N], const int (&j)[N],
                                      double (&v)[N]) {
  if (g.ident) {
#pragma unroll
    for (int u = 0; u < N; ++u)
      v[u] = (g.tr ? i[u] == j[u] + g.diag : j[u] == i[u] + g.diag) ? 1.0 : 0.0;
  } else if (g.f64) {
    const HLU_G double* p = gptr<const double>(g.ptr);
#pragma unroll
    for (int u = 0; u < N; ++u) v[u] = p[(int64_t)i[u] * g.si + (int64_t)j[u] * g.sj];
  } else {
    const HLU_G float* p = gptr<const float>(g.ptr);
    float f[N];
#pragma unroll
    for (int u = 0; u < N; ++u) f[u] = p[(int64_t)i[u] * g.si + (int64_t)j[u] * g.sj];
#pragma unroll
    for (int u = 0; u < N; ++u) v[u] = (double)f[u];
  }
}
template <int N>
__device__ __forceinline__ void gstore(const GView& g, const int (&i)[N], const int (&j)[N],
                                       const bool (&ok)[N], const double (&v)[N]) {
  if (g.f64) {
    HLU_G double* p = gptr<double>(g.ptr);
#pragma unroll
    for (int u = 0; u < N; ++u)
      if (ok[u]) p[(int64_t)i[u] * g.si + (int64_t)j[u] * g.sj] = v[u];
  } else {
    HLU_G float* p = gptr<float>(g.ptr);
#pragma unroll
    for (int u = 0; u < N; ++u)
      if (ok[u]) p[(int64_t)i[u] * g.si + (int64_t)j[u] * g.sj] = (float)v[u];
  }
}

// Staging of operand tiles into LDS with one memory round trip per tile.
// dst[a][b] = view(ri, cj) where map(a, b, ri, cj) returns whether the
// element is inside the operand (else it is staged as zero and (ri, cj) must
// still name an element inside the panel).  64 x 32 tiles:
template <class F>
__device__ __forceinline__ void stage_64x32(double (*dst)[33], const GView& g, F map) {
  int ri[8], cj[8];
  bool ok[8];
  double v[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int e = threadIdx.x + NT * u;
    ok[u] = map(e % 64, e / 64, ri[u], cj[u]);
  }
  gload(g, ri, cj, v);
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int e = threadIdx.x + NT * u;
    dst[e % 64][e / 64] = ok[u] ? v[u] : 0.0;
  }
}
// 32 x 64 tiles
template <class F>
__device__ __forceinline__ void stage_32x64(double (*dst)[65], const GView& g, F map) {
  int ri[8], cj[8];
  bool ok[8];
  double v[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int e = threadIdx.x + NT * u;
    ok[u] = map(e % 32, e / 32, ri[u], cj[u]);
  }
  gload(g, ri, cj, v);
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int e = threadIdx.x + NT * u;
    dst[e % 32][e / 32] = ok[u] ? v[u] : 0.0;
  }
}
// Y[r0 + ti + 16u][c0 + tj + 16v] += s * acc[u][v] within h x w (h, w >= 1):
// all loads first, then all stores (a store could alias a later load
// otherwise, and every element would cost a round trip)
__device__ __forceinline__ void tile_update(const PRef& Y, int r0, int c0, int h, int w, int ti,
                                            int tj, double s, const double (&acc)[4][4],
                                            bool ow = false) {
  const GView g = gview(Y);
  int ri[16], cj[16];
  bool ok[16];
  double v[16];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = ti + 16 * u, j = tj + 16 * q;
      ok[4 * u + q] = i < h && j < w;
      ri[4 * u + q] = r0 + min(i, h - 1);
      cj[4 * u + q] = c0 + min(j, w - 1);
    }
  if (ow) {
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = 0.0;
  } else {
    gload(g, ri, cj, v);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) v[4 * u + q] += s * acc[u][q];
  gstore(g, ri, cj, ok, v);
}

// cross-lane helpers (64-wide wavefronts)
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// FP64 matrix-core step D += A B with A 16 x 4 and B 4 x 16 (one wavefront):
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16], and its four
// results are D[l / 16 + 4r][l % 16], r = 0..3.
typedef double v4d __attribute__((ext_vector_type(4)));
__device__ __forceinline__ v4d mfma16x16x4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// FP32 matrix-core step D += A B with A 16 x 4 and B 4 x 16 (one
// wavefront): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16], and
// its four results are D[4 (l / 16) + r][l % 16], r = 0..3 (the f64 step
// above interleaves the result rows differently).
typedef float v4f __attribute__((ext_vector_type(4)));
__device__ __forceinline__ v4f mfma16x16x4f(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// FP32 counterparts of gload / gstore (mixed precision): FP64 storage is
// rounded to FP32 as it is loaded, an identity panel is evaluated.  The
// index rules of gload apply (every index inside the panel).
template <int N>
__device__ __forceinline__ void gloadf(const GView& g, const int (&i)[N], const int (&j)[N],
                                       float (&v)[N]) {
  if (g.ident) {
#pragma unroll
    for (int u = 0; u < N; ++u)
      v[u] = (g.tr ? i[u] == j[u] + g.diag : j[u] == i[u] + g.diag) ? 1.0f : 0.0f;
  } else if (g.f64) {
    const HLU_G double* p = gptr<const double>(g.ptr);
    double d[N];
#pragma unroll
    for (int u = 0; u < N; ++u) d[u] = p[(int64_t)i[u] * g.si + (int64_t)j[u] * g.sj];
#pragma unroll
    for (int u = 0; u < N; ++u) v[u] = (float)d[u];
  } else {
    const HLU_G float* p = gptr<const float>(g.ptr);
#pragma unroll
    for (int u = 0; u < N; ++u) v[u] = p[(int64_t)i[u] * g.si + (int64_t)j[u] * g.sj];
  }
}
template <int N>
__device__ __forceinline__ void gstoref(const GView& g, const int (&i)[N], const int (&j)[N],
                                        const bool (&ok)[N], const float (&v)[N]) {
  HLU_G float* p = gptr<float>(g.ptr);
#pragma unroll
  for (int u = 0; u < N; ++u)
    if (ok[u]) p[(int64_t)i[u] * g.si + (int64_t)j[u] * g.sj] = v[u];
}

// per-op record {model flops, algorithmic bytes, rank-capacity hit, rank,
// start tick, end tick, stack width, 0} (ticks of the constant-rate wall
// clock, written by thread 0)
__device__ __forceinline__ void put_cost(const Op& op, double flops, double bytes,
                                         double cap_hit = 0.0, double rank = 0.0,
                                         double width = 0.0, double detail = 0.0) {
  if (op.cost && threadIdx.x == 0) {
    HLU_G double* c = gptr<double>(op.cost);
    c[0] = flops;
    c[1] = bytes;
    c[2] = cap_hit;
    c[3] = rank;
    c[5] = (double)wall_clock64();
    c[6] = width;
    c[7] = detail;
  }
}

// an op's start time, taken as it starts and stored in its record once the
// op has run (a store at the start would wait for the loads in flight)
__device__ __forceinline__ void put_start(const Op& op, long long t0) {
  if (op.cost && threadIdx.x == 0) gptr<double>(op.cost)[4] = (double)t0;
}

// one step of a wave argmax (largest value, smallest index among equals)
// through a DPP lane permutation; lanes outside row_mask keep their own
template <int CTRL, int RM>
__device__ __forceinline__ void amax_dpp(double& v, int& ix) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(v), __double2loint(v), CTRL, RM, 0xf,
                                             false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(v), __double2hiint(v), CTRL, RM, 0xf,
                                             false);
  const int i2 = __builtin_amdgcn_update_dpp(ix, ix, CTRL, RM, 0xf, false);
  const double v2 = __hiloint2double(hi, lo);
  if (v2 > v || (v2 == v && i2 < ix)) {
    v = v2;
    ix = i2;
  }
}

// wave-wide argmax; the result (read from lane 63) is wave-uniform
__device__ __forceinline__ void wave_argmax(double& v, int& ix) {
  amax_dpp<0xB1, 0xf>(v, ix);    // quad_perm [1,0,3,2]
  amax_dpp<0x4E, 0xf>(v, ix);    // quad_perm [2,3,0,1]
  amax_dpp<0x141, 0xf>(v, ix);   // row_half_mirror
  amax_dpp<0x140, 0xf>(v, ix);   // row_mirror: every lane holds its row's result
  amax_dpp<0x142, 0xa>(v, ix);   // row_bcast:15 into rows 1 and 3
  amax_dpp<0x143, 0xc>(v, ix);   // row_bcast:31 into rows 2 and 3: lane 63 holds all
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  ix = __builtin_amdgcn_readlane(ix, 63);
  v = __hiloint2double(hi, lo);
}

// ---------------------------------------------------------------- getrf
// Right-looking unblocked LU with partial pivoting of one b x b leaf
// (b <= 64) held in LDS; pivot = first row of the largest |a_ik|.
// Contraction is disabled so that the elimination rounds exactly like the
// textbook update a - l*u.
#define LDS_GETRF (64 * 65 * 8 + 16)
__device__ void d_getrf(const Op& op) {
#pragma clang fp contract(off)
  char* const smem = hlu_lds;
  const PRef A = op.p[0];
  const int b = A.rows;
  double (*a)[65] = reinterpret_cast<double (*)[65]>(smem);
  int& s_piv = reinterpret_cast<int*>(smem + 64 * 65 * 8)[0];
  int& s_info = reinterpret_cast<int*>(smem + 64 * 65 * 8)[1];
  const int tid = threadIdx.x;
  HLU_G double* g = gptr<double>(A.ptr);
  for (int e = tid; e < b * b; e += NT) {
    int i = e % b, j = e / b;
    a[i][j] = g[i + (size_t)j * A.ld];
  }
  if (tid == 0) s_info = 0;
  HLU_G int32_t* piv = gptr<int32_t>(op.p[1].ptr);
  __syncthreads();
  for (int k = 0; k < b; ++k) {
    if (tid < 64) {
      // first row of the largest |a_ik| (DPP argmax, exact compare)
      double v = (tid >= k && tid < b) ? fabs(a[tid][k]) : -1.0;
      int ix = tid;
      wave_argmax(v, ix);
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
    {
      // rank-one update: lane i holds row i, wavefront w the columns
      // k + 1 + w, k + 5 + w, ... (no index division per element)
      const int i = tid & 63, w = tid >> 6;
      if (i > k && i < b) {
        const double l = a[i][k];
        for (int j = k + 1 + w; j < b; j += 4) {
          const double prod = l * a[k][j];
          a[i][j] = a[i][j] - prod;
        }
      }
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
// (OP_TRSM_U) with the factored b x b leaf p0 (b <= 64).
#define LDS_TRSM (64 * 65 * 8 + 64 * 8 + 64 * 4)
// Leaf solves on the columns of Y (b <= 64 rows): TRSM_L Y := L^{-1} P Y
// (unit lower, LAPACK-style row interchanges), TRSM_UT Y := U^{-T} Y,
// TRSM_U Y := U^{-1} Y.  The leaf sits in LDS (rows >= b hold zeros); the
// columns are solved with one lane per row (trsm_cols), without barriers.
// Columns of the leaf solve with one lane per row: lane i of wavefront w
// holds row i of columns w + 4(q0 + t), t < NC, and step k takes x_k of
// every column from lane k (a readlane), then updates the rows below (L,
// U^T) or above (U) with one multiply-add per column.  The arithmetic per
// entry is that of the eight-lane substitution.
template <int TYPE, int NC>
__device__ __forceinline__ void trsm_cols(const GView& gy, const double (*l)[65],
                                          const double* dinv, const int* pm, int b, int c,
                                          int q0) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ncw = (c - w + 3) >> 2;
  const int nq = min(NC, ncw - q0);
  const int il = min(lane, b - 1);
  int ri[NC], cj[NC];
  bool ok[NC];
  double v[NC];
#pragma unroll
  for (int t = 0; t < NC; ++t) {
    ri[t] = TYPE == OP_TRSM_L ? pm[il] : il;
    cj[t] = w + 4 * (q0 + min(t, nq - 1));
  }
  gload(gy, ri, cj, v);
  if (TYPE == OP_TRSM_U) {
    double lk = l[lane][b - 1];
    for (int k = b - 1; k >= 0; --k) {
      const double lnext = l[lane][k > 0 ? k - 1 : 0];
      const double dk = dinv[k];
#pragma unroll
      for (int t = 0; t < NC; ++t) {
        const double xk = readlane_d(v[t], k) * dk;
        v[t] = lane == k ? xk : (lane < k ? v[t] - lk * xk : v[t]);
      }
      lk = lnext;
    }
  } else {
    double lk = TYPE == OP_TRSM_UT ? l[0][lane] : l[lane][0];
    for (int k = 0; k < b; ++k) {
      const int kn = k + 1 < b ? k + 1 : k;
      const double lnext = TYPE == OP_TRSM_UT ? l[kn][lane] : l[lane][kn];
      if (TYPE == OP_TRSM_L) {
#pragma unroll
        for (int t = 0; t < NC; ++t) {
          const double xk = readlane_d(v[t], k);
          v[t] = (lane > k && lane < b) ? v[t] - lk * xk : v[t];
        }
      } else {
        const double dk = dinv[k];
#pragma unroll
        for (int t = 0; t < NC; ++t) {
          const double xk = readlane_d(v[t], k) * dk;
          v[t] = lane == k ? xk : ((lane > k && lane < b) ? v[t] - lk * xk : v[t]);
        }
      }
      lk = lnext;
    }
  }
#pragma unroll
  for (int t = 0; t < NC; ++t) {
    ok[t] = lane < b && t < nq;
    ri[t] = il;
  }
  gstore(gy, ri, cj, ok, v);
}
// The same column solve on an FP32 panel (mixed precision) in FP32
// arithmetic: the leaf's entries are rounded to FP32 as they are read, and
// x_k crosses lanes as one 32-bit readlane.
template <int TYPE, int NC>
__device__ __forceinline__ void trsm_cols_f32(const GView& gy, const double (*l)[65],
                                              const double* dinv, const int* pm, int b, int c,
                                              int q0) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ncw = (c - w + 3) >> 2;
  const int nq = min(NC, ncw - q0);
  const int il = min(lane, b - 1);
  int ri[NC], cj[NC];
  bool ok[NC];
  float v[NC];
#pragma unroll
  for (int t = 0; t < NC; ++t) {
    ri[t] = TYPE == OP_TRSM_L ? pm[il] : il;
    cj[t] = w + 4 * (q0 + min(t, nq - 1));
  }
  gloadf(gy, ri, cj, v);
  if (TYPE == OP_TRSM_U) {
    float lk = (float)l[lane][b - 1];
    for (int k = b - 1; k >= 0; --k) {
      const float lnext = (float)l[lane][k > 0 ? k - 1 : 0];
      const float dk = (float)dinv[k];
#pragma unroll
      for (int t = 0; t < NC; ++t) {
        const float xk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[t]), k)) * dk;
        v[t] = lane == k ? xk : (lane < k ? v[t] - lk * xk : v[t]);
      }
      lk = lnext;
    }
  } else {
    float lk = (float)(TYPE == OP_TRSM_UT ? l[0][lane] : l[lane][0]);
    for (int k = 0; k < b; ++k) {
      const int kn = k + 1 < b ? k + 1 : k;
      const float lnext = (float)(TYPE == OP_TRSM_UT ? l[kn][lane] : l[lane][kn]);
      if (TYPE == OP_TRSM_L) {
#pragma unroll
        for (int t = 0; t < NC; ++t) {
          const float xk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[t]), k));
          v[t] = (lane > k && lane < b) ? v[t] - lk * xk : v[t];
        }
      } else {
        const float dk = (float)dinv[k];
#pragma unroll
        for (int t = 0; t < NC; ++t) {
          const float xk =
              __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[t]), k)) * dk;
          v[t] = lane == k ? xk : ((lane > k && lane < b) ? v[t] - lk * xk : v[t]);
        }
      }
      lk = lnext;
    }
  }
#pragma unroll
  for (int t = 0; t < NC; ++t) {
    ok[t] = lane < b && t < nq;
    ri[t] = il;
  }
  gstoref(gy, ri, cj, ok, v);
}
template <int TYPE>
__device__ __forceinline__ void trsm_lanes_f32(const GView& gy, const double (*l)[65],
                                               const double* dinv, const int* pm, int b, int c) {
  const int ncw = (c + 3) >> 2;
  if (ncw <= 2) {
    if ((threadIdx.x >> 6) < c) trsm_cols_f32<TYPE, 2>(gy, l, dinv, pm, b, c, 0);
  } else if (ncw <= 4) {
    trsm_cols_f32<TYPE, 4>(gy, l, dinv, pm, b, c, 0);
  } else {
    const int w = threadIdx.x >> 6, mine = (c - w + 3) >> 2;
    for (int q0 = 0; q0 < mine; q0 += 8) trsm_cols_f32<TYPE, 8>(gy, l, dinv, pm, b, c, q0);
  }
}
template <int TYPE>
__device__ __forceinline__ void trsm_lanes(const GView& gy, const double (*l)[65],
                                           const double* dinv, const int* pm, int b, int c) {
  const int ncw = (c + 3) >> 2;   // columns of wavefront 0 (the most)
  if (ncw <= 2) {
    if ((threadIdx.x >> 6) < c) trsm_cols<TYPE, 2>(gy, l, dinv, pm, b, c, 0);
  } else if (ncw <= 4) {
    trsm_cols<TYPE, 4>(gy, l, dinv, pm, b, c, 0);
  } else {
    const int w = threadIdx.x >> 6, mine = (c - w + 3) >> 2;
    for (int q0 = 0; q0 < mine; q0 += 8) trsm_cols<TYPE, 8>(gy, l, dinv, pm, b, c, q0);
  }
}

__device__ __forceinline__ void trsm_body(const Op& op) {
  char* const smem = hlu_lds;
  const PRef L = op.p[0];
  const PRef Y = op.p[1];
  const int b = L.rows;
  const int c = pcols(Y);
  const int type = op.type;
  double (*l)[65] = reinterpret_cast<double (*)[65]>(smem);
  double* dinv = reinterpret_cast<double*>(smem + 64 * 65 * 8);
  int* pm = reinterpret_cast<int*>(smem + 64 * 65 * 8 + 64 * 8);
  const int tid = threadIdx.x;
  {
    const HLU_G double* g = gptr<const double>(L.ptr);
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + NT * u, i = e & 63, j = e >> 6;
      v[u] = (i < b && j < b) ? g[i + (size_t)j * L.ld] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + NT * u, i = e & 63, j = e >> 6;
      l[i][j] = v[u];
    }
  }
  if (tid < 64) {
    if (type == OP_TRSM_L) {
      // row permutation of the interchanges applied in order: lane i holds
      // the source row of position i
      const HLU_G int32_t* piv = gptr<const int32_t>(op.p[2].ptr);
      const int pk = tid < b ? piv[tid] : tid;
      int pr = tid;
      for (int k = 0; k < b; ++k) {
        const int p = __builtin_amdgcn_readlane(pk, k);
        const int vk = __builtin_amdgcn_readlane(pr, k), vp = __builtin_amdgcn_readlane(pr, p);
        pr = tid == k ? vp : (tid == p ? vk : pr);
      }
      pm[tid] = pr;
    }
  }
  __syncthreads();
  if (type != OP_TRSM_L && tid < b) dinv[tid] = 1.0 / l[tid][tid];
  __syncthreads();
  const GView gy = gview(Y);
  if (b > 0 && c > 0) {
    if (Y.dt == DT_F32) {
      if (type == OP_TRSM_L) trsm_lanes_f32<OP_TRSM_L>(gy, l, dinv, pm, b, c);
      else if (type == OP_TRSM_UT) trsm_lanes_f32<OP_TRSM_UT>(gy, l, dinv, pm, b, c);
      else trsm_lanes_f32<OP_TRSM_U>(gy, l, dinv, pm, b, c);
    } else {
      if (type == OP_TRSM_L) trsm_lanes<OP_TRSM_L>(gy, l, dinv, pm, b, c);
      else if (type == OP_TRSM_UT) trsm_lanes<OP_TRSM_UT>(gy, l, dinv, pm, b, c);
      else trsm_lanes<OP_TRSM_U>(gy, l, dinv, pm, b, c);
    }
  }
  const double es = Y.dt == DT_F64 ? 8.0 : 4.0;
  put_cost(op, (double)b * b * c, 8.0 * b * b / 2 + 2.0 * es * b * c);
}

// ---------------------------------------------------------------- panel products
// p3 += d0 * op(M) p2.  Dense M: tiles of 64 x 64 outputs with 32-deep LDS
// slabs.  Low-rank M = A B^T: T = B^T X (k x c) in LDS, then Y += d0 A T.
#define LDS_PGEMM_WIDE (64 * 33 * 8 + 32 * 65 * 8 + 64 * 65 * 8)
// narrow products: dense (M chunk 64 x 65, X chunk 64 x 17, partials 4 x 64 x 17)
// and low-rank (B chunk 64 x 33, X chunk 64 x 17, T 32 x 17, A tile 64 x 33,
// partials 4 x 64 x 17 = 8 x 32 x 17)
#define PGN_DENSE_DBL (64 * 65 + 64 * 17 + 4 * 64 * 17)
#define PGN_LR_DBL (64 * 33 + 64 * 17 + 32 * 17 + 64 * 33 + 4 * 64 * 17)
#define LDS_PGEMM_NARROW ((PGN_DENSE_DBL > PGN_LR_DBL ? PGN_DENSE_DBL : PGN_LR_DBL) * 8)
#define LDS_PGEMM (LDS_PGEMM_WIDE > LDS_PGEMM_NARROW ? LDS_PGEMM_WIDE : LDS_PGEMM_NARROW)

// R x C tile of a panel view held in registers (R * C / NT values per
// thread; consecutive lanes take consecutive rows, so column-major panels
// load coalesced).  load() reads rows a0 .. a0 + h - 1 and columns
// b0 .. b0 + w - 1 (h, w >= 1; lanes beyond them read a clamped element),
// put() stores the tile to LDS with zeros outside h x w.
template <int R, int C>
struct TileRegs {
  static constexpr int N = R * C / NT;
  double v[N];
  __device__ __forceinline__ void load(const GView& g, int a0, int b0, int h, int w) {
    int ri[N], cj[N];
#pragma unroll
    for (int u = 0; u < N; ++u) {
      const int e = threadIdx.x + NT * u;
      ri[u] = a0 + min(e % R, h - 1);
      cj[u] = b0 + min(e / R, w - 1);
    }
    gload(g, ri, cj, v);
  }
  template <int LD>
  __device__ __forceinline__ void put(double* dst, int h, int w) const {
#pragma unroll
    for (int u = 0; u < N; ++u) {
      const int e = threadIdx.x + NT * u, a = e % R, b = e / R;
      dst[a * LD + b] = (a < h && b < w) ? v[u] : 0.0;
    }
  }
};

// Sum of the four wavefronts' 64 x 16 partials (red[g][row][col], ld 17)
// plus the old values, stored to rows r0 .. r0 + h - 1, columns 0 .. w - 1
// of Y.  Thread t owns row t % 64, columns t / 64 + 4u (the layout of
// TileRegs<64, 16>).
__device__ __forceinline__ void narrow_finish(const GView& gy, const double* red, int r0, int h,
                                              int w, double sg, const double (&old)[4]) {
  const int a = threadIdx.x & 63;
  int ri[4], cj[4];
  bool ok[4];
  double out[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int b = (threadIdx.x >> 6) + 4 * u;
    const double s = red[a * 17 + b] + red[(64 + a) * 17 + b] + red[(128 + a) * 17 + b] +
                     red[(192 + a) * 17 + b];
    out[u] = old[u] + sg * s;
    ok[u] = a < h && b < w;
    ri[u] = r0 + min(a, h - 1);
    cj[u] = min(b, w - 1);
  }
  gstore(gy, ri, cj, ok, out);
}

// Y += sg * op(M) X for at most 16 columns.  Output tiles of 64 x 16; lane
// (ti, tj) of wavefront g holds rows ti + 16u, columns tj + 4v, and takes
// the inner indices 16g .. 16g + 15 of each 64-deep chunk; the four
// partials meet in LDS.  The old values of the tile and the first chunk
// are loaded together.
__device__ __forceinline__ void pgemm_narrow_dense(const Op& op, const PRef& X, const PRef& Y,
                                                   int m, int c, double sg, bool ow) {
  double* const sm = reinterpret_cast<double*>(hlu_lds);
  double* const sx = sm + 64 * 65;
  double* const red = sx + 64 * 17;
  const GView gm = gview(op.p[0], op.i1 != 0), gx = gview(X), gy = gview(Y);
  const int r = X.rows;
  const int tid = threadIdx.x, g = tid >> 6, ti = tid & 15, tj = (tid >> 4) & 3;
  for (int r0 = 0; r0 < m; r0 += 64) {
    const int h = min(64, m - r0);
    TileRegs<64, 16> yo;
    if (ow) {
#pragma unroll
      for (int u = 0; u < 4; ++u) yo.v[u] = 0.0;
    } else {
      yo.load(gy, r0, 0, h, c);
    }
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
    for (int k0 = 0; k0 < r; k0 += 64) {
      const int d = min(64, r - k0);
      TileRegs<64, 64> mt;
      TileRegs<64, 16> xt;
      mt.load(gm, r0, k0, h, d);
      xt.load(gx, k0, 0, d, c);
      mt.put<65>(sm, h, d);
      xt.put<17>(sx, d, c);
      __syncthreads();
      const int kb = 16 * g, ke = min(kb + 16, d);
      for (int kk = kb; kk < ke; ++kk) {
        double av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) av[u] = sm[(ti + 16 * u) * 65 + kk];
#pragma unroll
        for (int v = 0; v < 4; ++v) bv[v] = sx[kk * 17 + tj + 4 * v];
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
      for (int v = 0; v < 4; ++v) red[(g * 64 + ti + 16 * u) * 17 + tj + 4 * v] = acc[u][v];
    __syncthreads();
    narrow_finish(gy, red, r0, h, c, sg, yo.v);
    __syncthreads();
  }
}

// Y += sg * A (B^T X) for at most 16 columns and rank k <= 32 (A: m x k,
// B: r x k).  T = B^T X: lane (ta, tb) of group q (eight groups of 32
// lanes) holds T rows ta + 8u, columns tb + 4v over the rows 8q .. 8q + 7
// of each 64-row chunk, the next chunk loading while the current one is
// multiplied; the eight partials meet in LDS.  Then Y += sg A T tile by
// tile as in the dense case (wavefront g takes rank indices 8g .. 8g + 7),
// the first tile's A rows and old values loading with the first chunk and
// every later tile's while the previous one is computed.
__device__ __forceinline__ void pgemm_narrow_lr(const PRef& A, const PRef& B, const PRef& X,
                                                const PRef& Y, int m, int c, int k, double sg,
                                                bool ow) {
  double* const sb = reinterpret_cast<double*>(hlu_lds);
  double* const sx = sb + 64 * 33;
  double* const st = sx + 64 * 17;
  double* const sa = st + 32 * 17;
  double* const red = sa + 64 * 33;
  const GView ga = gview(A), gb = gview(B), gx = gview(X), gy = gview(Y);
  const int r = X.rows;
  const int tid = threadIdx.x;
  TileRegs<64, 32> at;
  TileRegs<64, 16> yo;
  at.load(ga, 0, 0, min(64, m), k);
  if (ow) {
#pragma unroll
    for (int u = 0; u < 4; ++u) yo.v[u] = 0.0;
  } else {
    yo.load(gy, 0, 0, min(64, m), c);
  }
  {
    const int q = tid >> 5, ta = tid & 7, tb = (tid >> 3) & 3;
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
    TileRegs<64, 32> bt;
    TileRegs<64, 16> xt;
    if (r > 0) {
      bt.load(gb, 0, 0, min(64, r), k);
      xt.load(gx, 0, 0, min(64, r), c);
    }
    for (int k0 = 0; k0 < r; k0 += 64) {
      const int d = min(64, r - k0);
      bt.put<33>(sb, d, k);
      xt.put<17>(sx, d, c);
      __syncthreads();
      if (k0 + 64 < r) {
        bt.load(gb, k0 + 64, 0, min(64, r - k0 - 64), k);
        xt.load(gx, k0 + 64, 0, min(64, r - k0 - 64), c);
      }
      const int ib = 8 * q, ie = min(ib + 8, d);
      for (int i = ib; i < ie; ++i) {
        double av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) av[u] = sb[i * 33 + ta + 8 * u];
#pragma unroll
        for (int v = 0; v < 4; ++v) bv[v] = sx[i * 17 + tb + 4 * v];
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
      for (int v = 0; v < 4; ++v) red[(q * 32 + ta + 8 * u) * 17 + tb + 4 * v] = acc[u][v];
    __syncthreads();
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      const int e = tid + NT * w, a = e & 31, b = e >> 5;
      double s = 0.0;
#pragma unroll
      for (int q2 = 0; q2 < 8; ++q2) s += red[(q2 * 32 + a) * 17 + b];
      st[a * 17 + b] = s;
    }
    __syncthreads();
  }
  const int g = tid >> 6, ti = tid & 15, tj = (tid >> 4) & 3;
  for (int r0 = 0; r0 < m; r0 += 64) {
    const int h = min(64, m - r0);
    at.put<33>(sa, h, k);
    __syncthreads();
    double old[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) old[u] = yo.v[u];
    if (r0 + 64 < m) {
      at.load(ga, r0 + 64, 0, min(64, m - r0 - 64), k);
      if (!ow) yo.load(gy, r0 + 64, 0, min(64, m - r0 - 64), c);
    }
    double o[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) o[u][v] = 0.0;
    const int kb = 8 * g, ke = min(kb + 8, k);
    for (int kk = kb; kk < ke; ++kk) {
      double av[4], tv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) av[u] = sa[(ti + 16 * u) * 33 + kk];
#pragma unroll
      for (int v = 0; v < 4; ++v) tv[v] = st[kk * 17 + tj + 4 * v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) o[u][v] += av[u] * tv[v];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[(g * 64 + ti + 16 * u) * 17 + tj + 4 * v] = o[u][v];
    __syncthreads();
    narrow_finish(gy, red, r0, h, c, sg, old);
    __syncthreads();
  }
}

// ---- FP32 panel products (mixed precision: the output panel is FP32)
// Y[:, c0:c0+c) += sg A (B^T X[:, c0:c0+c)) for rank k <= 32 (A: m x k,
// B: r x k, X: r x ., Y: m x ., c <= 16; FP32 storage, FP64 storage rounded
// to FP32 on load), on the FP32 matrix cores with FP32 accumulation:
//  1. T^T = X^T B over the rows in 64-row chunks staged in LDS: wavefront g
//     takes the rows 16g .. 16g + 15 of each chunk (one or two 16 x 16 tiles
//     of T^T), the next chunk loads while the current one is multiplied, and
//     the four partials meet in LDS;
//  2. Y^T = T^T A^T by 16-row tiles of Y (tile t to wavefront t % 4): A's
//     rows are read straight from memory in the operand layout (sixteen
//     consecutive rows of one column per load) and Y is updated in place.
#define PGF_LR_FLT (64 * 33 + 64 * 17 + 4 * 16 * 33 + 16 * 33)
__device__ __forceinline__ void pgemm_lr_f32(const PRef& A, const PRef& B, const PRef& X,
                                             const PRef& Y, int m, int c0, int c, int k,
                                             float sg, bool ow) {
  float* const sb = reinterpret_cast<float*>(hlu_lds);   // [64][33]: B chunk
  float* const sx = sb + 64 * 33;                        // [64][17]: X chunk
  float* const red = sx + 64 * 17;                       // [4][16][33]: partials
  float* const st = red + 4 * 16 * 33;                   // [16][33]: T^T
  const GView ga = gview(A), gb = gview(B), gx = gview(X), gy = gview(Y);
  const int r = X.rows;
  const int tid = threadIdx.x, g = tid >> 6, l = tid & 63, lo = l & 15, hi = l >> 4;
  {
    v4f acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    float pb[8], px[4];
    auto fetch = [&](int r0) {
      int ri[8], cb[8], rx[4], cx[4];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = tid + NT * u;
        ri[u] = min(r0 + (e & 63), r - 1);
        cb[u] = min(e >> 6, k - 1);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = tid + NT * u;
        rx[u] = min(r0 + (e & 63), r - 1);
        cx[u] = c0 + min(e >> 6, c - 1);
      }
      gloadf(gb, ri, cb, pb);
      gloadf(gx, rx, cx, px);
    };
    if (r > 0) fetch(0);
    for (int r0 = 0; r0 < r; r0 += 64) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = tid + NT * u, i = e & 63, j = e >> 6;
        sb[i * 33 + j] = (r0 + i < r && j < k) ? pb[u] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = tid + NT * u, i = e & 63, j = e >> 6;
        sx[i * 17 + j] = (r0 + i < r && j < c) ? px[u] : 0.f;
      }
      __syncthreads();
      if (r0 + 64 < r) fetch(r0 + 64);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = 16 * g + 4 * q + hi;
        const float a = sx[row * 17 + lo];
        acc0 = mfma16x16x4f(a, sb[row * 33 + lo], acc0);
        if (k > 16) acc1 = mfma16x16x4f(a, sb[row * 33 + 16 + lo], acc1);
      }
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      red[(g * 16 + 4 * hi + q) * 33 + lo] = acc0[q];
      red[(g * 16 + 4 * hi + q) * 33 + 16 + lo] = acc1[q];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = tid + NT * u, i = e >> 5, j = e & 31;
      st[i * 33 + j] = red[i * 33 + j] + red[(16 + i) * 33 + j] + red[(32 + i) * 33 + j] +
                       red[(48 + i) * 33 + j];
    }
    __syncthreads();
  }
  const int nk = (k + 3) >> 2;
  for (int t = g; 16 * t < m; t += 4) {
    const int row = 16 * t + lo;
    int ri[8], cj[8], yr[4], yc[4];
    bool ok[4];
    float av[8], yv[4];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      ri[q] = min(row, m - 1);
      cj[q] = min(4 * q + hi, k - 1);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      yr[q] = min(row, m - 1);
      yc[q] = c0 + min(4 * hi + q, c - 1);
      ok[q] = row < m && 4 * hi + q < c;
    }
    gloadf(ga, ri, cj, av);
    if (ow) {
#pragma unroll
      for (int q = 0; q < 4; ++q) yv[q] = 0.f;
    } else {
      gloadf(gy, yr, yc, yv);
    }
    v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (q < nk) {
        const int kk = 4 * q + hi;
        acc = mfma16x16x4f(st[lo * 33 + kk], kk < k ? av[q] : 0.f, acc);
      }
#pragma unroll
    for (int q = 0; q < 4; ++q) yv[q] += sg * acc[q];
    gstoref(gy, yr, yc, ok, yv);
  }
}

// Y[:, c0:c0+c) += sg op(M) X[:, c0:c0+c) for a dense M (m x r, any
// storage, rounded to FP32) and an FP32 output panel, c <= 16: per 64-row
// block of Y and 64-deep chunk of the inner dimension, the X chunk is staged
// in LDS and wavefront g multiplies the rows 16g .. 16g + 15, reading M's
// rows straight from memory in the operand layout (Y^T = X^T M^T).
#define PGF_DENSE_FLT (64 * 17)
__device__ __forceinline__ void pgemm_dense_f32(const Op& op, const PRef& X, const PRef& Y,
                                                int m, int c0, int c, float sg, bool ow) {
  float* const sx = reinterpret_cast<float*>(hlu_lds);   // [64][17]
  const GView gm = gview(op.p[0], op.i1 != 0), gx = gview(X), gy = gview(Y);
  const int r = X.rows;
  const int tid = threadIdx.x, g = tid >> 6, l = tid & 63, lo = l & 15, hi = l >> 4;
  for (int r0 = 0; r0 < m; r0 += 64) {
    const int row = r0 + 16 * g + lo;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    int yr[4], yc[4];
    bool ok[4];
    float yv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      yr[q] = min(row, m - 1);
      yc[q] = c0 + min(4 * hi + q, c - 1);
      ok[q] = row < m && 4 * hi + q < c;
    }
    if (ow) {
#pragma unroll
      for (int q = 0; q < 4; ++q) yv[q] = 0.f;
    } else {
      gloadf(gy, yr, yc, yv);
    }
    for (int k0 = 0; k0 < r; k0 += 64) {
      const int d = min(64, r - k0);
      float px[4], mv[16];
      int rx[4], cx[4], mi[16], mj[16];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = tid + NT * u;
        rx[u] = k0 + min(e & 63, d - 1);
        cx[u] = c0 + min(e >> 6, c - 1);
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        mi[q] = min(row, m - 1);
        mj[q] = k0 + min(4 * q + hi, d - 1);
      }
      gloadf(gx, rx, cx, px);
      gloadf(gm, mi, mj, mv);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = tid + NT * u, i = e & 63, j = e >> 6;
        sx[i * 17 + j] = (i < d && j < c) ? px[u] : 0.f;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int kk = 4 * q + hi;
        acc = mfma16x16x4f(sx[kk * 17 + lo], kk < d ? mv[q] : 0.f, acc);
      }
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) yv[q] += sg * acc[q];
    gstoref(gy, yr, yc, ok, yv);
  }
}

__device__ __forceinline__ void pgemm_body(const Op& op) {
  char* const smem = hlu_lds;
  const PRef X = op.p[2];
  const PRef Y = op.p[3];
  const double sg = op.d0;
  const int tid = threadIdx.x;
  const int cy = pcols(Y), cx = pcols(X);
  const int kl = op.i0 == 0 ? 0 : pcols(op.p[0]);
  const int c = min(cy, cx);
  const int m = Y.rows;
  const double esx = X.dt == DT_F64 ? 8.0 : 4.0;
  // i2 bit 0: the first product into a fresh panel overwrites it (Y := ...)
  // instead of accumulating; its old values are then neither read nor counted
  const bool ow = (op.i2 & 1) != 0;
  const double esy = (Y.dt == DT_F64 ? 8.0 : 4.0) * (ow ? 0.5 : 1.0);
  if (ow && op.i0 == 1 && kl == 0) {
    // a rank-0 operand: the product is zero, and the fresh panel must still
    // be written (later products accumulate into it)
    const GView gy = gview(Y);
    const int tot = m * cy;
    for (int e0 = 0; e0 < tot; e0 += NT * 4) {
      int ri[4], cj[4];
      bool ok[4];
      double z[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = min(e0 + threadIdx.x + NT * u, tot - 1);
        ri[u] = e % m;
        cj[u] = e / m;
        ok[u] = e0 + (int)threadIdx.x + NT * u < tot;
        z[u] = 0.0;
      }
      gstore(gy, ri, cj, ok, z);
    }
    put_cost(op, 0.0, esy * m * cy);
    return;
  }
  if (Y.dt == DT_F32 && (op.i0 == 0 || kl <= 32)) {
    // FP32 output panel (mixed precision): FP32 arithmetic on the matrix
    // cores, 16 columns at a time
    const int r = X.rows;
    const bool tr = op.i1 != 0;
    if (c > 0 && m > 0 && (op.i0 == 0 || kl > 0)) {
      for (int c0 = 0; c0 < c; c0 += 16) {
        const int cw = min(16, c - c0);
        if (op.i0 == 0)
          pgemm_dense_f32(op, X, Y, m, c0, cw, (float)sg, ow);
        else
          pgemm_lr_f32(tr ? op.p[1] : op.p[0], tr ? op.p[0] : op.p[1], X, Y, m, c0, cw, kl,
                       (float)sg, ow);
        __syncthreads();
      }
    }
    if (op.i0 == 0) {
      put_cost(op, 2.0 * m * r * c, 8.0 * m * r + esx * r * c + 2.0 * esy * m * c);
    } else {
      const double esm = op.p[0].dt == DT_F64 ? 8.0 : 4.0;
      put_cost(op, 2.0 * (double)kl * c * (r + m),
               esm * (double)kl * (r + m) + esx * r * c + 2.0 * esy * m * c);
    }
    return;
  }
  if (c <= 16 && (op.i0 == 0 || kl <= 32)) {
    const int r = X.rows;
    if (op.i0 == 0) {
      if (c > 0 && m > 0) pgemm_narrow_dense(op, X, Y, m, c, sg, ow);
      put_cost(op, 2.0 * m * r * c, 8.0 * m * r + esx * r * c + 2.0 * esy * m * c);
    } else {
      const bool tr = op.i1 != 0;
      if (c > 0 && m > 0 && kl > 0)
        pgemm_narrow_lr(tr ? op.p[1] : op.p[0], tr ? op.p[0] : op.p[1], X, Y, m, c, kl, sg, ow);
      const double esm = op.p[0].dt == DT_F64 ? 8.0 : 4.0;
      put_cost(op, 2.0 * (double)kl * c * (r + m),
               esm * (double)kl * (r + m) + esx * r * c + 2.0 * esy * m * c);
    }
    return;
  }
  double (*sa)[33] = reinterpret_cast<double (*)[33]>(smem);
  double (*sb)[65] = reinterpret_cast<double (*)[65]>(smem + 64 * 33 * 8);
  double (*st)[65] = reinterpret_cast<double (*)[65]>(smem + 64 * 33 * 8 + 32 * 65 * 8);
  const int ti = tid % 16, tj = tid / 16;   // 16 x 16 threads, 4 x 4 outputs each
  if (op.i0 == 0) {
    const GView gm = gview(op.p[0], op.i1 != 0), gx = gview(X);
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
          stage_64x32(sa, gm, [&](int i, int kk, int& a, int& b) {
            a = r0 + min(i, h - 1);
            b = k0 + min(kk, d - 1);
            return i < h && kk < d;
          });
          stage_32x64(sb, gx, [&](int kk, int j, int& a, int& b) {
            a = k0 + min(kk, d - 1);
            b = c0 + min(j, w - 1);
            return kk < d && j < w;
          });
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
        tile_update(Y, r0, c0, h, w, ti, tj, sg, acc, ow);
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
  const int k = kl;
  const int r = X.rows;
  const double esm = U.dt == DT_F64 ? 8.0 : 4.0;
  const GView ga = gview(A), gb = gview(B, true), gx = gview(X);
  for (int c0 = 0; c0 < (k > 0 ? c : 0); c0 += 64) {
    const int w = min(64, c - c0);
    // T = B^T X  (k x w), k <= 64
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
    for (int k0 = 0; k0 < r; k0 += 32) {
      const int d = min(32, r - k0);
      // i: rank index, kk: row of B
      stage_64x32(sa, gb, [&](int i, int kk, int& a, int& b) {
        a = min(i, k - 1);
        b = k0 + min(kk, d - 1);
        return i < k && kk < d;
      });
      stage_32x64(sb, gx, [&](int kk, int j, int& a, int& b) {
        a = k0 + min(kk, d - 1);
        b = c0 + min(j, w - 1);
        return kk < d && j < w;
      });
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
      stage_64x32(sa, ga, [&](int i, int kk, int& a, int& b) {
        a = r0 + min(i, h - 1);
        b = min(kk, k - 1);
        return i < h && kk < k;
      });
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
        stage_64x32(sa, ga, [&](int i, int kk, int& a, int& b) {
          a = r0 + min(i, h - 1);
          b = min(32 + kk, k - 1);
          return i < h && 32 + kk < k;
        });
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
      tile_update(Y, r0, c0, h, w, ti, tj, sg, o, ow);
    }
    __syncthreads();
  }
  put_cost(op, 2.0 * (double)k * c * (r + m),
           esm * (double)k * (r + m) + esx * r * c + 2.0 * esy * m * c);
}

// ---------------------------------------------------------------- dense update
// p0 (FP64 dense, m x n) -= p1 p2^T
#define LDS_ADDD (64 * 33 * 8 + 32 * 65 * 8)
// Mixed precision, FP32 factors X (m x k) and Y (n x k): the product X Y^T
// runs on the FP32 matrix cores with FP32 accumulation (C^T = Y X^T in
// 16 x 16 tiles; wavefront g takes the columns 16g .. 16g + 15 of each
// 64 x 64 block of C and its four row tiles, reading both factors straight
// from memory in the operand layout), and is subtracted from the FP64
// block in FP64.
__device__ __forceinline__ void addd_f32(const PRef& C, const PRef& X, const PRef& Y, int m,
                                         int n, int k) {
  const GView gx = gview(X), gy = gview(Y), gc = gview(C);
  const int tid = threadIdx.x, g = tid >> 6, l = tid & 63, lo = l & 15, hi = l >> 4;
  for (int c0 = 0; c0 < n; c0 += 64) {
    const int col0 = c0 + 16 * g;
    for (int r0 = 0; r0 < m; r0 += 64) {
      if (col0 >= n) continue;
      v4f acc[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = (v4f){0.f, 0.f, 0.f, 0.f};
      for (int k0 = 0; k0 < k; k0 += 32) {
        float yv[8], xv[4][8];
        int yi[8], yj[8], xi[8], xj[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          yi[q] = min(col0 + lo, n - 1);
          yj[q] = min(k0 + 4 * q + hi, k - 1);
          xj[q] = yj[q];
        }
        gloadf(gy, yi, yj, yv);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
          for (int q = 0; q < 8; ++q) xi[q] = min(r0 + 16 * t + lo, m - 1);
          gloadf(gx, xi, xj, xv[t]);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (k0 + 4 * q < k) {
            const bool in = k0 + 4 * q + hi < k;
            const float a = in ? yv[q] : 0.f;
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[t] = mfma16x16x4f(a, in ? xv[t][q] : 0.f, acc[t]);
          }
      }
      int ci[16], cj[16];
      bool ok[16];
      double v[16];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = r0 + 16 * t + lo, j = col0 + 4 * hi + q;
          ci[4 * t + q] = min(i, m - 1);
          cj[4 * t + q] = min(j, n - 1);
          ok[4 * t + q] = i < m && j < n;
        }
      gload(gc, ci, cj, v);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) v[4 * t + q] -= (double)acc[t][q];
      gstore(gc, ci, cj, ok, v);
    }
  }
}
// FP64 factors (plain FP64 mode, dense near-field panels): C^T = Y X^T on
// the FP64 matrix cores in 16 x 16 tiles, wavefront g taking the columns
// 16g .. 16g + 15 of each 64 x 64 block of C and its four row tiles, both
// factors read straight from memory in the operand layout (sixteen
// consecutive rows of one column per load for column-major panels).
__device__ __forceinline__ void addd_f64(const PRef& C, const PRef& X, const PRef& Y, int m,
                                         int n, int k) {
  const GView gx = gview(X), gy = gview(Y), gc = gview(C);
  const int tid = threadIdx.x, g = tid >> 6, l = tid & 63, lo = l & 15, hi = l >> 4;
  for (int c0 = 0; c0 < n; c0 += 64) {
    const int col0 = c0 + 16 * g;
    for (int r0 = 0; r0 < m; r0 += 64) {
      if (col0 >= n) continue;
      v4d acc[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = (v4d){0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < k; k0 += 16) {
        double yv[4], xv[4][4];
        int yi[4], yj[4], xi[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          yi[q] = min(col0 + lo, n - 1);
          yj[q] = min(k0 + 4 * q + hi, k - 1);
        }
        gload(gy, yi, yj, yv);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
          for (int q = 0; q < 4; ++q) xi[q] = min(r0 + 16 * t + lo, m - 1);
          gload(gx, xi, yj, xv[t]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (k0 + 4 * q < k) {
            const bool in = k0 + 4 * q + hi < k;
            const double a = in ? yv[q] : 0.0;
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[t] = mfma16x16x4(a, in ? xv[t][q] : 0.0, acc[t]);
          }
      }
      int ci[16], cj[16];
      bool ok[16];
      double v[16];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = r0 + 16 * t + lo, j = col0 + hi + 4 * q;
          ci[4 * t + q] = min(i, m - 1);
          cj[4 * t + q] = min(j, n - 1);
          ok[4 * t + q] = i < m && j < n;
        }
      gload(gc, ci, cj, v);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) v[4 * t + q] -= acc[t][q];
      gstore(gc, ci, cj, ok, v);
    }
  }
}
__device__ __forceinline__ void addd_body(const Op& op) {
  char* const smem = hlu_lds;
  const PRef C = op.p[0], X = op.p[1], Y = op.p[2];
  const int m = C.rows, n = C.cols;
  const int k = pcols(X);
  if (X.dt == DT_F32 && Y.dt == DT_F32 && X.kind == PK_MAT && Y.kind == PK_MAT) {
    if (m > 0 && n > 0 && k > 0) addd_f32(C, X, Y, m, n, k);
    put_cost(op, 2.0 * m * n * k, 16.0 * m * n + 4.0 * (double)k * (m + n));
    return;
  }
  if (X.dt == DT_F64 && Y.dt == DT_F64 && X.kind == PK_MAT && Y.kind == PK_MAT) {
    if (m > 0 && n > 0 && k > 0) addd_f64(C, X, Y, m, n, k);
    put_cost(op, 2.0 * m * n * k, 16.0 * m * n + 8.0 * (double)k * (m + n));
    return;
  }
  double (*sa)[33] = reinterpret_cast<double (*)[33]>(smem);
  double (*sb)[65] = reinterpret_cast<double (*)[65]>(smem + 64 * 33 * 8);
  const int tid = threadIdx.x;
  const int ti = tid % 16, tj = tid / 16;
  const GView gx = gview(X), gy = gview(Y, true);
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
        stage_64x32(sa, gx, [&](int i, int kk, int& a, int& b) {
          a = r0 + min(i, h - 1);
          b = k0 + min(kk, d - 1);
          return i < h && kk < d;
        });
        stage_32x64(sb, gy, [&](int kk, int j, int& a, int& b) {
          a = k0 + min(kk, d - 1);
          b = c0 + min(j, w - 1);
          return kk < d && j < w;
        });
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
      tile_update(C, r0, c0, h, w, ti, tj, -1.0, acc);
    }
  }
  const double es = X.dt == DT_F64 ? 8.0 : 4.0;
  put_cost(op, 2.0 * m * n * k, 16.0 * m * n + es * (double)k * (m + n));
}

// ---------------------------------------------------------------- zero
__device__ __forceinline__ void zero_body(const Op& op) {
  const PRef Z = op.p[0];
  const int tot = Z.rows * Z.cols;
  const GView g = gview(Z);
  if (g.f64) {
    HLU_G double* p = gptr<double>(g.ptr);
    for (int e = threadIdx.x; e < tot; e += NT)
      p[(int64_t)(e % Z.rows) * g.si + (int64_t)(e / Z.rows) * g.sj] = 0.0;
  } else {
    HLU_G float* p = gptr<float>(g.ptr);
    for (int e = threadIdx.x; e < tot; e += NT)
      p[(int64_t)(e % Z.rows) * g.si + (int64_t)(e / Z.rows) * g.sj] = 0.0f;
  }
  put_cost(op, 0.0, (Z.dt == DT_F64 ? 8.0 : 4.0) * tot);
}

// ---------------------------------------------------------------- truncation
// C = U V^T (rank kc) minus a list of low-rank terms X_t Y_t^T (X_t placed at
// row xo_t of C, Y_t at row yo_t, zero elsewhere).  The terms are taken in
// passes whose stacked width K = kc + sum k_t stays <= 64 (live ranks read at
// run time); every pass replaces C by the best approximation of
// [U, -X_a, ..., -X_b] [V, Y_a, ..., Y_b]^T:
//   1. Gram matrices Gx = Xs^T Xs, Gy = Ys^T Ys in FP64, both sides in one
//      sweep over row chunks of 64 (4x4 blocks per thread over row groups);
//   2. column balancing so that |x_j| = |y_j|;
//   3. pivoted Cholesky Gx = Pi_x R^T R Pi_x^T and Gy = Pi_y S^T S Pi_y^T,
//      one wavefront each (concurrently, no barriers), stopping at pivots
//      below 1e-14 of the largest diagonal;
//   4. M = R S^T and its singular values and left singular vectors W by
//      one-sided Jacobi on the columns of M;
//   5. rank choice (fixed, or the smallest k with discarded Frobenius norm
//      <= eps |Sig|, capped);
//   6. Tx = D Pi_x R11^{-1} W_k and Ty = D^{-1} R^T W_k: with
//      Qx = Xs D Pi_x R11^{-1} the new factors are U = Qx W_k and
//      V = Ys D^{-1} R^T W_k = C^T Qx W_k, so U V^T = Qx W_k W_k^T Qx^T C is
//      the projection of C onto its leading k left singular vectors (the
//      best rank-k approximation, without the right singular vectors);
//   7. U := Xs Tx, V := Ys Ty streamed in place (each row chunk is read
//      before it is written).
#define KM 64
#define TMAX 16

// Stacked column j of one side: element i is sign * base[(i - r0) * stride]
// for r0 <= i < r0 + rows and zero elsewhere; an identity column (ident)
// holds a single one at row r0 + irow.
// Stacked column j of one side, resolved once per pass: element i (a row of
// the stacked panel) lies at base0 + i * sbytes for lo <= i < hi and is zero
// elsewhere; an identity column holds a single one at row irow.  flags: bit
// 0 FP64 storage, bit 1 identity, bit 2 negated.  Read as two 16-byte words.
struct __align__(16) ColDesc {
  uint64_t base0;
  int32_t sbytes, lo, hi, irow;
  uint32_t flags, pad;
};
static_assert(sizeof(ColDesc) == 32, "column descriptors are read as two 16-byte words");

struct TruncShared {
  double lv[2][KM];         // pivot rows broadcast by the two Cholesky waves (16-byte aligned)
  double gx[KM][KM + 1];    // Gx -> R (row s: pivot step s) / X-side apply chunk
  double gy[KM][KM + 1];    // Y-side Gram chunk / Gy -> S / Jacobi buffer / Ty
  double m[KM][KM + 1];     // X-side Gram chunk / M -> W Sig -> Tx
  double z[KM][KM + 1];     // Gram partials / W_k / Y-side apply chunk
  ColDesc cd[2][KM];
  double dsc[KM];
  double sig[KM];
  double nrm[2][KM];        // squared column norms by position (Jacobi, double-buffered)
  double rinv[KM];          // 1 / R11[i][i]
  double red[4];
  Term tm[TMAX];
  int px[KM], py[KM], ord[KM];
  int8_t colt[KM], colj[KM];
  int tw[TMAX];             // live widths of the candidate terms of a pass
  int rx, ry, k, capped, K, kc, te, jcur, jsweeps;
  double mnorm;
};

// sum over aligned groups of g consecutive lanes (g = 8, 16, 32 or 64)
__device__ __forceinline__ double group_sum(double v, int g) {
  v += dpp_d<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);   // row_half_mirror
  if (g >= 16) v += dpp_d<0x140>(v);   // row_mirror
  if (g >= 32) v += __shfl_xor(v, 16);
  if (g >= 64) v += __shfl_xor(v, 32);
  return v;
}

// sum over the whole wavefront by DPP alone (row sums, then the row
// broadcasts carry rows 0-2 into row 3); the result is wave-uniform
template <int CTRL, int RM>
__device__ __forceinline__ double dpp_dm(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, RM, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, RM, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0xB1>(v);          // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);          // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);         // row_half_mirror
  v += dpp_d<0x140>(v);         // row_mirror: every lane holds its row's sum
  v += dpp_dm<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_dm<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3: lane 63 holds all
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// v[p] for a wave-uniform p (a branch tree, no per-element selects)
#define HLU_C8(C, b) C(b) C(b + 1) C(b + 2) C(b + 3) C(b + 4) C(b + 5) C(b + 6) C(b + 7)
#define HLU_C64(C) HLU_C8(C, 0) HLU_C8(C, 8) HLU_C8(C, 16) HLU_C8(C, 24) \
  HLU_C8(C, 32) HLU_C8(C, 40) HLU_C8(C, 48) HLU_C8(C, 56)
__device__ __forceinline__ double pick64(const double (&v)[KM], int p) {
  double r = 0.0;
  switch (p) {
#define HLU_PICK(i) case i: r = v[i]; break;
    HLU_C64(HLU_PICK)
#undef HLU_PICK
    default: break;
  }
  return r;
}
// Wave-wide choice of the lane with the largest candidate value v >= 0
// (scaled by inv_scale into [0, 1]) through one 32-bit key per lane: the
// float bits of the scaled value with the low six bits replaced by
// 63 - lane, so each step is a single unsigned max.  Values that agree in
// their leading 17 mantissa bits count as equal and go to the lowest lane.
// Returns the lane (wave-uniform), or -1 when no lane is a candidate.
template <int CTRL, int RM>
__device__ __forceinline__ uint32_t umax_dpp(uint32_t k) {
  const uint32_t o = (uint32_t)__builtin_amdgcn_update_dpp((int)k, (int)k, CTRL, RM, 0xf, false);
  return o > k ? o : k;
}
__device__ __forceinline__ int wave_argmax_key(double v, bool cand, double inv_scale) {
  const int lane = threadIdx.x & 63;
  const float f = (float)(v * inv_scale);
  uint32_t key = (cand && f > 0.0f) ? ((__float_as_uint(f) & ~63u) | (uint32_t)(63 - lane)) : 0u;
  key = umax_dpp<0xB1, 0xf>(key);    // quad_perm [1,0,3,2]
  key = umax_dpp<0x4E, 0xf>(key);    // quad_perm [2,3,0,1]
  key = umax_dpp<0x141, 0xf>(key);   // row_half_mirror
  key = umax_dpp<0x140, 0xf>(key);   // row_mirror
  key = umax_dpp<0x142, 0xa>(key);   // row_bcast:15
  key = umax_dpp<0x143, 0xc>(key);   // row_bcast:31: lane 63 holds the maximum
  key = (uint32_t)__builtin_amdgcn_readlane((int)key, 63);
  return key ? 63 - (int)(key & 63u) : -1;
}

__device__ __forceinline__ double block_sum(TruncShared& sh, double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) sh.red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double s = sh.red[0] + sh.red[1] + sh.red[2] + sh.red[3];
  __syncthreads();
  return s;
}

__device__ __forceinline__ double block_max(TruncShared& sh, double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) sh.red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double s = fmax(fmax(sh.red[0], sh.red[1]), fmax(sh.red[2], sh.red[3]));
  __syncthreads();
  return s;
}

// descriptors of the K stacked columns of both sides ([U, -X..] and [V, Y..])
__device__ __forceinline__ void trunc_coldesc(TruncShared& sh, const PRef& U, const PRef& V) {
  const int K = sh.K, kc = sh.kc;
  for (int e = threadIdx.x; e < 2 * K; e += NT) {
    const int side = e >= K, j = e - side * K;
    // fields copied one by one (a reference chosen between two local
    // panels would force both into private memory)
    uint64_t ptr;
    int32_t ld, rows, r0, cj, sg;
    uint8_t dt, trans, kind;
    if (j < kc) {
      ptr = side ? V.ptr : U.ptr;
      ld = side ? V.ld : U.ld;
      rows = side ? V.rows : U.rows;
      dt = side ? V.dt : U.dt;
      trans = side ? V.trans : U.trans;
      kind = side ? V.kind : U.kind;
      r0 = 0;
      cj = j;
      sg = 1;
    } else {
      const Term& t = sh.tm[sh.colt[j]];
      const PRef& F = side ? t.Y : t.X;   // LDS: no copy
      ptr = F.ptr;
      ld = F.ld;
      rows = F.rows;
      dt = F.dt;
      trans = F.trans;
      kind = F.kind;
      r0 = side ? t.yo : t.xo;
      cj = sh.colj[j];
      sg = side ? 1 : -1;
    }
    ColDesc d;
    const int64_t es = dt == DT_F64 ? 8 : 4;
    const int64_t sb = (trans ? (int64_t)ld : 1) * es;
    // the panel's row ii is stacked row r0 + ii
    d.base0 = ptr + (uint64_t)((trans ? (int64_t)cj : (int64_t)cj * ld) * es) -
              (uint64_t)((int64_t)r0 * sb);
    d.sbytes = (int32_t)sb;
    d.lo = r0;
    d.hi = r0 + rows;
    d.irow = r0 + cj - ld;   // identity: (ii, cj) is one iff cj == ii + ld
    d.flags = (dt == DT_F64 ? 1u : 0u) | (kind == PK_IDENT ? 2u : 0u) | (sg < 0 ? 4u : 0u);
    d.pad = 0;
    sh.cd[side][j] = d;
  }
}

// Word that column reads of absent and identity entries load instead of
// panel memory (so every load of a chunk is issued unconditionally).
__device__ __align__(16) uint32_t hlu_zero_words[4];

// rows [r0, r0 + 64) of both stacked panels into d0 (X side) and d1 (Y
// side).  Lane i of wavefront w takes row r0 + i of the stacked columns
// w + 4u (u = 0..15) of each side.  The descriptors are read four columns at
// a time, addresses are formed with selects (absent and identity entries
// read a zero word), and all 32 word loads of a side are in flight before
// the first is converted: one memory round trip per side and chunk.
__device__ __forceinline__ void trunc_load2(TruncShared& sh, double (*d0)[KM + 1],
                                            double (*d1)[KM + 1], int r0, int m, int n, int K) {
  const int tid = threadIdx.x, i = tid & 63, w = tid >> 6;
  const int row = r0 + i;
  const uint64_t zero = (uint64_t)hlu_zero_words;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    double (*d)[KM + 1] = side ? d1 : d0;
    const uint4* cd = reinterpret_cast<const uint4*>(&sh.cd[side][0]);
    uint32_t lo[16], hi[16], fl[16];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      uint4 a[4], b[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = w + 4 * (4 * g + v);
        const int jj = j < K ? j : 0;
        a[v] = cd[2 * jj];
        b[v] = cd[2 * jj + 1];
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int u = 4 * g + v, j = w + 4 * u;
        const uint64_t base0 = (uint64_t)a[v].x | ((uint64_t)a[v].y << 32);
        const int sb = (int)a[v].z, clo = (int)a[v].w, chi = (int)b[v].x, irow = (int)b[v].y;
        const uint32_t f = b[v].z;
        const bool in = j < K && row >= clo && row < chi;
        const bool mem = in && !(f & 2u);
        const uint64_t addr = base0 + (uint64_t)((int64_t)row * sb);
        const uint64_t pl = mem ? addr : zero;
        const uint64_t ph = (mem && (f & 1u)) ? addr + 4 : zero;
        lo[u] = *gptr<const uint32_t>(pl);
        hi[u] = *gptr<const uint32_t>(ph);
        fl[u] = (f & 5u) | ((in && (f & 2u) && row == irow) ? 2u : 0u) | (j < K ? 8u : 0u);
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      double v = (fl[u] & 1u) ? __hiloint2double((int)hi[u], (int)lo[u])
                              : (double)__int_as_float((int)lo[u]);
      if (fl[u] & 2u) v = 1.0;
      if (fl[u] & 4u) v = -v;
      if (fl[u] & 8u) d[i][w + 4 * u] = v;
    }
  }
  (void)m;
  (void)n;
}

// Gram tiles of one wavefront: tile t = W, W + 2, ... of the NB (NB + 1) / 2
// 16 x 16 tiles on and above the diagonal, numbered row by row.  Each step
// of four rows reads the NB column blocks once and feeds the independent
// tiles back to back.
constexpr int gram_tile_row(int nb, int t) {
  int a = 0;
  while (t >= nb - a) {
    t -= nb - a;
    ++a;
  }
  return a;
}
constexpr int gram_tile_col(int nb, int t) {
  int a = 0;
  while (t >= nb - a) {
    t -= nb - a;
    ++a;
  }
  return a + t;
}
template <int NB, int W, int J>
__device__ __forceinline__ void gram_step(const double (&cv)[NB], v4d (&acc)[5]) {
  if constexpr (J < 5 && W + 2 * J < NB * (NB + 1) / 2) {
    constexpr int t = W + 2 * J;
    constexpr int a = gram_tile_row(NB, t), b = gram_tile_col(NB, t);
    acc[J] = mfma16x16x4(cv[a], cv[b], acc[J]);
    gram_step<NB, W, J + 1>(cv, acc);
  }
}
template <int NB, int W>
__device__ __forceinline__ void gram_tiles(double (*C)[KM + 1], int nq, v4d (&acc)[5]) {
  const int l = threadIdx.x & 63;
  // steps in groups of four, straight-line inside a group (the matrix-core
  // builtins are convergent, so the compiler does not unroll a loop with a
  // variable trip count); rows past the chunk's end are zero in LDS
  for (int q0 = 0; q0 < nq; q0 += 4) {
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
      const int i = 4 * (q0 + qq) + (l >> 4);
      double cv[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) cv[c] = C[i][16 * c + (l & 15)];
      gram_step<NB, W, 0>(cv, acc);
    }
  }
}

// Gx into gx and Gy into gy: threads 0-127 take the X side (chunks staged in
// m), threads 128-255 the Y side (chunks staged in gy).  The matrix cores
// form the 16 x 16 tiles on and above the diagonal (at most ten, dealt to
// the side's two wavefronts), four rows per step; the tiles above the
// diagonal are mirrored when written.
__device__ __forceinline__ void trunc_gram2(TruncShared& sh, int m, int n, int K) {
  const int tid = threadIdx.x;
  const int side = tid >> 7, w = (tid >> 6) & 1, l = tid & 63;
  const int rows_side = side ? n : m;
  double (*C)[KM + 1] = side ? sh.gy : sh.m;
  double (*G)[KM + 1] = side ? sh.gy : sh.gx;
  const int nb = (K + 15) >> 4, ntile = nb * (nb + 1) / 2;
  v4d acc[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) acc[j] = (v4d){0.0, 0.0, 0.0, 0.0};
  const int rows = max(m, n);
  for (int r0 = 0; r0 < rows; r0 += 64) {
    trunc_load2(sh, sh.m, sh.gy, r0, m, n, K);
    __syncthreads();
    const int nq = min(16, (rows_side - r0 + 3) >> 2);
    switch (nb * 2 + w) {
      case 2: gram_tiles<1, 0>(C, nq, acc); break;
      case 3: gram_tiles<1, 1>(C, nq, acc); break;
      case 4: gram_tiles<2, 0>(C, nq, acc); break;
      case 5: gram_tiles<2, 1>(C, nq, acc); break;
      case 6: gram_tiles<3, 0>(C, nq, acc); break;
      case 7: gram_tiles<3, 1>(C, nq, acc); break;
      case 8: gram_tiles<4, 0>(C, nq, acc); break;
      case 9: gram_tiles<4, 1>(C, nq, acc); break;
      default: break;
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const int t = w + 2 * j;
    if (t < ntile) {
      const int ta = 16 * gram_tile_row(nb, t), tb = 16 * gram_tile_col(nb, t);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = ta + (l >> 4) + 4 * r, b = tb + (l & 15);
        if (a < K && b < K) {
          G[a][b] = acc[j][r];
          if (ta != tb) G[b][a] = acc[j][r];
        }
      }
    }
  }
  __syncthreads();
}

// Pivoted Cholesky of the K x K matrix G by one wavefront; lane j keeps
// column j of the trailing matrix in registers.  On exit row s of G holds
// row s of R in stacked-column order (zero in the columns pivoted before
// step s), piv[0..r) are the pivots in order, piv[r..K) the remaining
// columns, and r is the numerical rank.  lv (64 doubles, 16-byte aligned)
// carries each step's row of R to every lane.
// Pivot of the next step from the trailing diagonal d (wave-uniform p and
// v = d[p]); false once the pivoted Cholesky stops: no candidate left, a
// pivot below 1e-14 of the largest initial diagonal, or (TRACE_STOP) a
// residual diagonal summing to at most trace_stop.
template <bool TRACE_STOP>
__device__ __forceinline__ bool pchol_pick(double d, bool alive, double dmax0, double inv_dmax0,
                                           double trace_stop, int& p, double& v) {
  // straight-line (no early exit), so that the caller's LDS reads issued
  // before it stay in flight across it
  bool ok = dmax0 > 0.0;
  if constexpr (TRACE_STOP) {
    // the squared distances of the remaining rows from the span of the
    // chosen ones
    const double trace = wave_sum(alive ? fmax(d, 0.0) : 0.0);
    ok = ok && trace > trace_stop;
  }
  p = wave_argmax_key(d, alive, inv_dmax0);
  v = readlane_d(d, p < 0 ? 0 : p);
  return ok && p >= 0 && v > 1e-14 * dmax0;
}

template <bool TRACE_STOP = false>
__device__ __forceinline__ void trunc_pchol_wave(double (*G)[KM + 1], double* lv, int* piv, int K,
                                                 int* r_out, double trace_stop = 0.0,
                                                 double* trace_out = nullptr) {
  const int lane = threadIdx.x & 63;
  const bool in = lane < K;
  double g[KM];
#pragma unroll
  for (int i = 0; i < KM; ++i) g[i] = (in && i < K) ? G[i][lane] : 0.0;
  double d = in ? G[lane][lane] : 0.0;
  double dmax0 = d;
  int dummy = lane;
  wave_argmax(dmax0, dummy);
  const double inv_dmax0 = dmax0 > 0.0 ? 1.0 / dmax0 : 0.0;
  bool alive = in;
  int r = 0, p = 0;
  double v = 0.0;
  bool go = pchol_pick<TRACE_STOP>(d, alive, dmax0, inv_dmax0, trace_stop, p, v);
  while (go) {
    // 1 / sqrt(v) by the hardware estimate and one Newton step, sqrt(v) from it
    double inv = __builtin_amdgcn_rsq(v);
    inv = inv * (1.5 - 0.5 * v * inv * inv);
    const double rp = v * inv;
    const double l = alive ? (lane == p ? rp : pick64(g, p) * inv) : 0.0;
    if (in) G[r][lane] = l;
    lv[lane] = l;
    if (lane == 0) piv[r] = p;
    if (lane == p) alive = false;
    d -= l * l;
    ++r;
    // rank-one update of the trailing columns (same wavefront: the loads
    // below see the stores above).  Straight-line over all 64 entries: lanes
    // at or beyond K hold l = 0, so their entries stay zero, and without a
    // branch per entry the reads are issued together.  Two halves of 32
    // rows keep the batch within the register budget of the inlined
    // executor; the next pivot, which needs only the diagonal, is chosen
    // while the first half's reads are in flight.
    const double2* l2 = reinterpret_cast<const double2*>(lv);
    double2 lr[KM / 4];
#pragma unroll
    for (int i = 0; i < KM / 2; i += 2) lr[i >> 1] = l2[i >> 1];
    go = pchol_pick<TRACE_STOP>(d, alive, dmax0, inv_dmax0, trace_stop, p, v);
#pragma unroll
    for (int i = 0; i < KM / 2; i += 2) {
      g[i] -= lr[i >> 1].x * l;
      g[i + 1] -= lr[i >> 1].y * l;
    }
#pragma unroll
    for (int i = 0; i < KM / 2; i += 2) lr[i >> 1] = l2[(KM / 2 + i) >> 1];
#pragma unroll
    for (int i = 0; i < KM / 2; i += 2) {
      g[KM / 2 + i] -= lr[i >> 1].x * l;
      g[KM / 2 + i + 1] -= lr[i >> 1].y * l;
    }
  }
  const unsigned long long mask = __ballot(alive);
  if (alive) piv[r + __popcll(mask & ((1ull << lane) - 1ull))] = lane;
  if (lane == 0) *r_out = r;
  if constexpr (TRACE_STOP) {
    const double trace = wave_sum(alive ? fmax(d, 0.0) : 0.0);
    if (lane == 0) *trace_out = trace;
  }
}

// Tx = D Pi_x R11^{-1} W_k into m (rows = stacked columns), W_k in z and
// R11[i][t] = gx[i][px[t]] (k <= 32).  One lane per row: lane t of
// wavefront w holds row t of columns w + 4q, q < NQ; step i takes every
// column's x_i from lane i by a readlane and updates the rows above it.
template <int NQ>
__device__ __forceinline__ void trunc_trsv_cols(TruncShared& sh, int rx, int K, int k) {
  const int t = threadIdx.x & 63, w = threadIdx.x >> 6;
  double v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int c = w + 4 * q;
    v[q] = (t < rx && c < k) ? sh.z[t][c] : 0.0;
  }
  for (int i = rx - 1; i >= 0; --i) {
    const int pi = sh.px[i];
    const double ri = sh.rinv[i];
    const double g = sh.gx[t][pi];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double xi = readlane_d(v[q], i) * ri;
      v[q] = t == i ? xi : (t < i ? v[q] - g * xi : v[q]);
    }
  }
  if (t < K) {
    const int row = sh.px[t];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int c = w + 4 * q;
      if (c < k) sh.m[row][c] = t < rx ? v[q] * sh.dsc[row] : 0.0;
    }
  }
}
__device__ __forceinline__ void trunc_trsv8(TruncShared& sh, int rx, int K, int k) {
  const int nq = (k + 3) >> 2;
  if (nq <= 2) trunc_trsv_cols<2>(sh, rx, K, k);
  else if (nq <= 4) trunc_trsv_cols<4>(sh, rx, K, k);
  else trunc_trsv_cols<8>(sh, rx, K, k);
}

// new rows of U (threads 0-127, Tx in m) and V (threads 128-255, Ty in gy),
// chunks staged in gx / z
// out^T tiles of one wavefront in the factor update: row blocks W and W + 2
// of the chunk, NCT column blocks; each step of four stacked columns reads
// the two row blocks of C and the NCT column blocks of T once.
template <int NCT>
__device__ __forceinline__ void apply_tiles(double (*C)[KM + 1], double (*T)[KM + 1], int K,
                                            int w, v4d (&acc)[2][2]) {
  const int l = threadIdx.x & 63;
  const int nq = (K + 3) >> 2;
  // steps in groups of four, straight-line inside a group (columns past K
  // enter as zeros)
  for (int q0 = 0; q0 < nq; q0 += 4)
#pragma unroll
  for (int qq = 0; qq < 4; ++qq) {
    const int kk = 4 * (q0 + qq) + (l >> 4);
    const bool in = kk < K;
    double cv[2], tv[NCT];
    // read unconditionally (kk < KM), then select: a conditional read would
    // become a branch with a wait of its own per read
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const double v = C[16 * (w + 2 * u) + (l & 15)][min(kk, KM - 1)];
      cv[u] = in ? v : 0.0;
    }
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      const double v = T[min(kk, KM - 1)][16 * c + (l & 15)];
      tv[c] = in ? v : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < NCT; ++c) acc[u][c] = mfma16x16x4(tv[c], cv[u], acc[u][c]);
  }
}

__device__ __forceinline__ void trunc_apply2(TruncShared& sh, const PRef& U, const PRef& V, int m,
                                             int n, int K, int k) {
  // per side and row chunk: out (64 x k) = C (64 x K) T (K x k), taken
  // transposed on the matrix cores (out^T = T^T C^T) so that the sixteen
  // lanes of a result register hold consecutive rows; the side's two
  // wavefronts take alternate 16-row blocks
  const int tid = threadIdx.x;
  const int side = tid >> 7, w = (tid >> 6) & 1, l = tid & 63;
  const int rows_side = side ? n : m;
  double (*C)[KM + 1] = side ? sh.z : sh.gx;
  double (*T)[KM + 1] = side ? sh.gy : sh.m;
  const GView g = gview(side ? V : U);
  const int rows = max(m, n);
  const int nct = (k + 15) >> 4;
  for (int r0 = 0; r0 < rows; r0 += 64) {
    trunc_load2(sh, sh.gx, sh.z, r0, m, n, K);
    __syncthreads();
    const int h = rows_side - r0;
    if (h > 0 && nct > 0) {
      v4d acc[2][2];
#pragma unroll
      for (int u = 0; u < 2; ++u) acc[u][0] = acc[u][1] = (v4d){0.0, 0.0, 0.0, 0.0};
      if (nct == 1) apply_tiles<1>(C, T, K, w, acc);
      else apply_tiles<2>(C, T, K, w, acc);
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          if (c < nct && 16 * (w + 2 * u) < h) {
            int ri[4], cj[4];
            bool ok[4];
            double o[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = 16 * (w + 2 * u) + (l & 15), col = 16 * c + (l >> 4) + 4 * r;
              ok[r] = row < h && col < k;
              ri[r] = r0 + min(row, h - 1);
              cj[r] = min(col, k - 1);
              o[r] = acc[u][c][r];
            }
            gstore(g, ri, cj, ok, o);
          }
        }
    }
    __syncthreads();
  }
}

// Physical column of Jacobi position p: consecutive positions land eight
// columns apart, so the pairs handled by one wavefront read and write
// disjoint LDS bank windows.
__device__ __forceinline__ int jphys(int p) { return ((p & 7) << 3) | (p >> 3); }

// One-sided Jacobi on at most 16 columns held in the registers of
// wavefront 0: lane l keeps column l & 15 at rows 4t + (l >> 4), t < T
// (rx <= 4T).  The columns stay in their lanes; round r of a sweep pairs
// them by the round-robin tournament on ncol (even) columns: column ncol-1
// meets column r and every other column c meets (2r - c) mod (ncol - 1).
// The partner's rows arrive by lane permutes, the inner product and the
// squared norms are reduced over the four row blocks by lane exchanges, and
// both lanes of a pair form the same rotation from the same values, so no
// round touches LDS.  Squared norms are recomputed at every sweep and
// carried through the rotations in between; sweeps stop once no pair had a
// squared cosine above stop.  The result goes back to m (columns by
// position, as the LDS version leaves them).
template <int T>
__device__ __forceinline__ void trunc_jacobi_reg(TruncShared& sh, int rx, int ncol, double ms,
                                                 double stop, int& sweeps_out) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    const int c = tid & 15, rb = tid >> 4;
    const bool col_in = c < ncol;
    double a[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int i = 4 * t + rb;
      a[t] = (col_in && i < rx) ? sh.m[i][jphys(c)] : 0.0;
    }
    const double tiny = 1e-30 * ms;
    const int nm1 = ncol - 1;
    int sweeps = 0;
    for (int sweep = 0; sweep < 30; ++sweep) {
      double al = 0.0;
#pragma unroll
      for (int t = 0; t < T; ++t) al += a[t] * a[t];
      al += __shfl_xor(al, 16);
      al += __shfl_xor(al, 32);
      double mu = 0.0;
      for (int r = 0; r < nm1; ++r) {
        int pc = c == nm1 ? r : (c == r ? nm1 : (2 * r - c + nm1) % nm1);
        if (!col_in) pc = c;
        const int src = (tid & 48) | pc;
        double b[T];
#pragma unroll
        for (int t = 0; t < T; ++t) b[t] = __shfl(a[t], src);
        const double be_ = __shfl(al, src);
        double ga = 0.0;
#pragma unroll
        for (int t = 0; t < T; ++t) ga += a[t] * b[t];
        ga += __shfl_xor(ga, 16);
        ga += __shfl_xor(ga, 32);
        // the pair (p, q), p < q, seen the same way from both of its lanes
        const bool first = c < pc;
        const double ap = first ? al : be_, aq = first ? be_ : al;
        double cs = 1.0, sn = 0.0, ap2 = ap, aq2 = aq;
        if (col_in && pc != c && ap > tiny && aq > tiny && ga * ga > 1e-30 * ap * aq) {
          mu = fmax(mu, ga * ga / (ap * aq));
          const double d = aq - ap, g2 = 2.0 * ga;
          const double rr = sqrt(d * d + g2 * g2), ad = fabs(d);
          const double y = 2.0 * rr * (rr + ad);
          double qy = __builtin_amdgcn_rsq(y);
          qy = qy * (1.5 - 0.5 * y * qy * qy);
          sn = (d >= 0.0 ? g2 : -g2) * qy;
          cs = (rr + ad) * qy;
          const double c2 = cs * cs, s2 = sn * sn, cg = 2.0 * cs * sn * ga;
          ap2 = c2 * ap - cg + s2 * aq;
          aq2 = s2 * ap + cg + c2 * aq;
        }
        // p' = cs p - sn q, q' = sn p + cs q
#pragma unroll
        for (int t = 0; t < T; ++t) a[t] = first ? cs * a[t] - sn * b[t] : sn * b[t] + cs * a[t];
        al = first ? ap2 : aq2;
      }
      ++sweeps;
      for (int o = 32; o > 0; o >>= 1) mu = fmax(mu, __shfl_xor(mu, o));
      if (!(mu > stop)) break;
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int i = 4 * t + rb;
      if (col_in && i < rx) sh.m[i][jphys(c)] = a[t];
    }
    if (tid == 0) sh.jsweeps = sweeps;
  }
  __syncthreads();
  sweeps_out = sh.jsweeps;
}

// One-sided Jacobi on the columns of M (rx rows, ry columns, initially
// position j = column j of m).  Round-robin ordering by the circle method:
// position 0 stays, positions 1..n-1 advance by one each round, position p
// pairs with n-1-p.  Each round reads one buffer and writes the rotated
// columns to their next positions in the other (m <-> gy); a group of grp
// lanes handles one pair, each lane at most 8 rows of both columns in
// registers.  Squared column norms (by position) are recomputed at every
// sweep and carried through the rotations in between, so a round reduces
// one inner product.  Sweeps stop once no pair had a squared cosine above
// stop.  At most 16 columns go to the register version above instead.
// Returns the buffer holding the result (0: m, 1: gy).
__device__ __forceinline__ int trunc_jacobi(TruncShared& sh, int rx, int ry, double ms,
                                            double stop, int& sweeps) {
  const int tid = threadIdx.x;
  const int ncol = ry + (ry & 1);
  sweeps = 0;
  if (ncol < 2 || rx <= 0 || !(ms > 0.0)) return 0;
  const int npair = ncol / 2, nm1 = ncol - 1;
  if (npair <= 8) {
    if (rx <= 16) trunc_jacobi_reg<4>(sh, rx, ncol, ms, stop, sweeps);
    else if (rx <= 32) trunc_jacobi_reg<8>(sh, rx, ncol, ms, stop, sweeps);
    else trunc_jacobi_reg<16>(sh, rx, ncol, ms, stop, sweeps);
    return 0;
  }
  int grp = 64;
  while (grp > 8 && grp * npair > NT) grp >>= 1;
  const int q = tid / grp, l = tid % grp;
  const bool act = q < npair;
  const int p0 = q, p1 = nm1 - q;                                    // this pair's positions
  const int n0 = q == 0 ? 0 : q + 1, n1 = q == 0 ? 1 : ncol - q;     // and the next ones
  const int f0 = jphys(p0), f1 = jphys(p1), g0 = jphys(n0), g1 = jphys(n1);
  const double tiny = 1e-30 * ms;
  int cur = 0;
  for (int sweep = 0; sweep < 30; ++sweep) {
    {
      double (*A)[KM + 1] = cur ? sh.gy : sh.m;
      const int j = tid >> 2, part = tid & 3;
      double s2 = 0.0;
      if (j < ncol) {
        const int fj = jphys(j);
        for (int i = part; i < rx; i += 4) s2 += A[i][fj] * A[i][fj];
      }
      s2 += dpp_d<0xB1>(s2);
      s2 += dpp_d<0x4E>(s2);
      if (part == 0 && j < ncol) sh.nrm[cur][j] = s2;
    }
    __syncthreads();
    double mu = 0.0;
    for (int round = 0; round < nm1; ++round) {
      if (act) {
        double (*S)[KM + 1] = cur ? sh.gy : sh.m;
        double (*D)[KM + 1] = cur ? sh.m : sh.gy;
        double ma[8], mb[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int i = l + grp * t;
          ma[t] = i < rx ? S[i][f0] : 0.0;
          mb[t] = i < rx ? S[i][f1] : 0.0;
        }
        const double al = sh.nrm[cur][p0], be = sh.nrm[cur][p1];
        double ga = 0.0;
#pragma unroll
        for (int t = 0; t < 8; ++t) ga += ma[t] * mb[t];
        ga = group_sum(ga, grp);
        double cs = 1.0, sn = 0.0, al2 = al, be2 = be;
        if (al > tiny && be > tiny && ga * ga > 1e-30 * al * be) {
          mu = fmax(mu, ga * ga / (al * be));
          // rotation zeroing the inner product of the pair:
          // c = sqrt((r + |d|) / 2r), s = sign(d) 2ga / sqrt(2r (r + |d|))
          const double d = be - al, g2 = 2.0 * ga;
          const double rr = sqrt(d * d + g2 * g2), ad = fabs(d);
          const double y = 2.0 * rr * (rr + ad);
          double qy = __builtin_amdgcn_rsq(y);
          qy = qy * (1.5 - 0.5 * y * qy * qy);
          sn = (d >= 0.0 ? g2 : -g2) * qy;
          cs = (rr + ad) * qy;
          const double c2 = cs * cs, s2 = sn * sn, cg = 2.0 * cs * sn * ga;
          al2 = c2 * al - cg + s2 * be;
          be2 = s2 * al + cg + c2 * be;
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int i = l + grp * t;
          if (i < rx) {
            D[i][g0] = cs * ma[t] - sn * mb[t];
            D[i][g1] = sn * ma[t] + cs * mb[t];
          }
        }
        if (l == 0) {
          sh.nrm[cur ^ 1][n0] = al2;
          sh.nrm[cur ^ 1][n1] = be2;
        }
      }
      __syncthreads();
      cur ^= 1;
    }
    ++sweeps;
    if (!(block_max(sh, mu) > stop)) break;
  }
  return cur;
}

#define LDS_TRUNC (sizeof(TruncShared))
__device__ __forceinline__ void d_trunc(const Op& op, int tune = 0) {
  char* const smem = hlu_lds;
  const PRef U = op.p[0], V = op.p[1];
  const Term* terms = reinterpret_cast<const Term*>(op.p[2].ptr) + op.i0;
  const int nterms = op.i1;
  const int cap = op.i2 & 0xffff, fixed = op.i2 >> 16;
  const double eps = op.d0;
  // sizes are the same for every thread: keep them in scalar registers
  const int m = __builtin_amdgcn_readfirstlane(U.rows);
  const int n = __builtin_amdgcn_readfirstlane(V.rows);
  TruncShared& sh = *reinterpret_cast<TruncShared*>(smem);
  const int tid = threadIdx.x, wid = tid >> 6;
  double flops = 0.0, bytes = 0.0;
  const double es = U.dt == DT_F64 ? 8.0 : 4.0;
  int capped_any = 0, Kmax = 0, passes = 0, sweeps_all = 0, rxmax = 0, rymax = 0;
  // widest stack of one pass (tuned per run; the first term of a pass is
  // always taken, so any width makes progress)
  const int kwide = (tune & 0xff) > 0 && (tune & 0xff) < KM ? (tune & 0xff) : KM;
  if (tid == 0) sh.te = 0;
  __syncthreads();
  for (;;) {
    // every thread reads the term cursor before thread 0 advances it
    const int te0 = sh.te;
    __syncthreads();
    if (te0 >= nterms) break;
    // choose this pass's terms and map the stacked columns: the candidate
    // terms and their live widths are read by one thread each, then
    // thread 0 takes terms while the stack fits (the first always)
    {
      const int cand = min(TMAX, nterms - te0);
      if (tid < cand) {
        const Term tt = terms[te0 + tid];
        sh.tm[tid] = tt;
        sh.tw[tid] = pcols(tt.X);
      } else if (tid == 64) {
        sh.kc = pcols(U);
      }
      __syncthreads();
      if (tid == 0) {
        int K = sh.kc, t = 0;
        while (t < cand) {
          const int w = sh.tw[t];
          if (t > 0 && K + w > kwide) break;
          K += w;
          ++t;
        }
        sh.K = K;
        sh.te = te0 + t;
        sh.capped = 0;
      }
      __syncthreads();
      // stacked column j of the terms: term t, column j - (kc + widths before t)
      for (int j = tid; j < KM; j += NT) {
        int c = j - sh.kc, t = 0;
        if (c >= 0 && j < sh.K) {
          while (c >= sh.tw[t]) {
            c -= sh.tw[t];
            ++t;
          }
          sh.colt[j] = (int8_t)t;
          sh.colj[j] = (int8_t)c;
        }
      }
    }
    __syncthreads();
    const int K = __builtin_amdgcn_readfirstlane(sh.K);
    Kmax = max(Kmax, K);
    trunc_coldesc(sh, U, V);
    __syncthreads();
    // 1. Gram matrices
    trunc_gram2(sh, m, n, K);
    // 2. balancing
    for (int j = tid; j < K; j += NT) {
      const double a = sh.gx[j][j], b = sh.gy[j][j];
      sh.dsc[j] = (a > 0.0 && b > 0.0) ? sqrt(sqrt(b / a)) : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < K * K; e += NT) {
      const int a = e % K, b = e / K;
      const double da = sh.dsc[a], db = sh.dsc[b];
      sh.gx[a][b] *= da * db;
      sh.gy[a][b] = (da > 0.0 && db > 0.0) ? sh.gy[a][b] / (da * db) : 0.0;
    }
    __syncthreads();
    // 3. pivoted Cholesky of both sides, one wavefront each
    if (wid == 0) trunc_pchol_wave(sh.gx, sh.lv[0], sh.px, K, &sh.rx);
    else if (wid == 1) trunc_pchol_wave(sh.gy, sh.lv[1], sh.py, K, &sh.ry);
    __syncthreads();
    const int rx = __builtin_amdgcn_readfirstlane(sh.rx);
    const int ry = __builtin_amdgcn_readfirstlane(sh.ry);
    // 4. M = R S^T (rows and columns in pivot order), |M|_F^2: 16 x 16 tiles
    // covering rx x ry on the matrix cores (wavefront w takes tiles w, w + 4,
    // ...), zeros everywhere else in the 64 x 64 buffer
    double msq = 0.0;
    {
      const int l = tid & 63;
      const int nbx = (rx + 15) >> 4, nby = (ry + 15) >> 4, nq = (K + 3) >> 2;
      for (int e = tid; e < KM * KM; e += NT) {
        const int i = e & 63, p = e >> 6;
        if (i >= 16 * nbx || p >= 16 * nby) sh.m[i][jphys(p)] = 0.0;
      }
      for (int t = wid; t < nbx * nby; t += 4) {
        const int i0 = 16 * (t % nbx), j0 = 16 * (t / nbx);
        v4d acc = {0.0, 0.0, 0.0, 0.0};
        for (int q0 = 0; q0 < nq; q0 += 4)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const int c = 4 * (q0 + qq) + (l >> 4);
          const bool in = c < K;
          const int cc = min(c, KM - 1);
          const double av = sh.gx[i0 + (l & 15)][cc], bv = sh.gy[j0 + (l & 15)][cc];
          acc = mfma16x16x4(in ? av : 0.0, in ? bv : 0.0, acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + (l >> 4) + 4 * r, j = j0 + (l & 15);
          const double v = (i < rx && j < ry) ? acc[r] : 0.0;
          sh.m[i][jphys(j)] = v;
          msq += v * v;
        }
      }
    }
    const double ms = block_sum(sh, msq);
    // 4b. for a tolerance-driven truncation, shrink the SVD to the part of M
    // that can matter: a pivoted Cholesky of G = M M^T, stopped once the
    // discarded rows of M (orthogonal to the kept ones) hold at most
    // (eps/4)^2 |M|_F^2, leaves L (rx x jc) with L L^T = M P M^T for an
    // orthogonal projector P.  The left singular vectors of L are those of
    // M P, and the discarded part is Frobenius-orthogonal to every
    // projection of M P, so its squared norm simply opens the tail of the
    // rank rule.  Squaring M is harmless at eps >= 1e-6 (FP64 Gram).
    int jc = ry;
    double tail0 = 0.0;
    const bool reduced = fixed == 0 && eps >= 1e-6 && rx > 8 && ry > 8;
    if (reduced) {
      {
        // G = M M^T (rx x rx): tiles on and above the diagonal, mirrored
        const int l = tid & 63;
        const int nb = (rx + 15) >> 4, ntl = nb * (nb + 1) / 2, nq = (ry + 3) >> 2;
        for (int t = wid; t < ntl; t += 4) {
          const int a0 = 16 * gram_tile_row(nb, t), b0 = 16 * gram_tile_col(nb, t);
          v4d acc = {0.0, 0.0, 0.0, 0.0};
          for (int q0 = 0; q0 < nq; q0 += 4)
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            const int j = 4 * (q0 + qq) + (l >> 4);
            const bool in = j < ry;
            const int fj = jphys(min(j, KM - 1));
            const double av = sh.m[a0 + (l & 15)][fj], bv = sh.m[b0 + (l & 15)][fj];
            acc = mfma16x16x4(in ? av : 0.0, in ? bv : 0.0, acc);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int a = a0 + (l >> 4) + 4 * r, b = b0 + (l & 15);
            if (a < rx && b < rx) {
              sh.gy[a][b] = acc[r];
              if (a0 != b0) sh.gy[b][a] = acc[r];
            }
          }
        }
      }
      __syncthreads();
      if (wid == 0)
        trunc_pchol_wave<true>(sh.gy, sh.lv[0], sh.py, rx, &sh.k, eps * eps * ms / 16.0,
                               &sh.mnorm);
      __syncthreads();
      jc = __builtin_amdgcn_readfirstlane(sh.k);
      tail0 = sh.mnorm;
      // L into the Jacobi buffer: column s of L is row s of the factored G
      for (int e = tid; e < rx * KM; e += NT) {
        const int i = e % rx, c = e / rx;
        sh.m[i][jphys(c)] = c < jc ? sh.gy[c][i] : 0.0;
      }
      __syncthreads();
    }
    // rotations stop at a cosine of 1e-3 eps (at most 1e-12): the singular
    // values then carry relative errors of order (1e-3 eps)^2, far below the
    // tolerance the rank rule resolves
    int sweeps;
    const double jstop = fixed == 0 ? fmax(1e-24, 1e-6 * eps * eps) : 1e-24;
    double (*MF)[KM + 1] = trunc_jacobi(sh, rx, jc, ms, jstop, sweeps) ? sh.gy : sh.m;
    passes += 1;
    sweeps_all += sweeps;
    rxmax = max(rxmax, rx);
    rymax = max(rymax, jc);
    // 5. singular values (column norms, by position; an odd ry has one zero
    // column more), descending order (stable), rank choice
    const int nr = rx > 0 ? jc : 0;
    const int npos = rx > 0 ? jc + (jc & 1) : 0;
    {
      const int j = tid >> 2, part = tid & 3;
      double s = 0.0;
      if (j < npos) {
        const int fj = jphys(j);
        for (int i = part; i < rx; i += 4) s += MF[i][fj] * MF[i][fj];
      }
      s += dpp_d<0xB1>(s);
      s += dpp_d<0x4E>(s);
      if (part == 0 && j < npos) sh.sig[j] = sqrt(s);
    }
    __syncthreads();
    for (int j = tid; j < npos; j += NT) {
      const double sj = sh.sig[j];
      int c = 0;
      for (int i = 0; i < npos; ++i) {
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
        double tot = tail0;
        for (int j = 0; j < npos; ++j) tot += sh.sig[j] * sh.sig[j];
        const double thr = eps * eps * tot;
        double tail = tail0;
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
    const int k = __builtin_amdgcn_readfirstlane(sh.k);
    capped_any |= sh.capped;
    // 6. W_k (normalised leading columns) into z, 1 / R11[i][i]; then
    // Tx = D Pi_x R11^{-1} W_k into m and Ty = D^{-1} R^T W_k into gy
    for (int e = tid; e < rx * k; e += NT) {
      const int i = e % rx, c = e / rx;
      const int j = sh.ord[c];
      const double sj = sh.sig[j];
      sh.z[i][c] = sj > 0.0 ? MF[i][jphys(j)] / sj : 0.0;
    }
    for (int i = tid; i < rx; i += NT) sh.rinv[i] = 1.0 / sh.gx[i][sh.px[i]];
    __syncthreads();
    trunc_trsv8(sh, rx, K, k);
    {
      const int tc = tid & 15, tk = tid >> 4;   // 4 stacked columns x 2 output columns
      double acc[4][2];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u][0] = acc[u][1] = 0.0;
      const int c20 = tc * 4, c0 = tk * 2;
      if (c0 < k) {
        for (int i = 0; i < rx; ++i) {
          double rv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) rv[u] = c20 + u < K ? sh.gx[i][c20 + u] : 0.0;
          const double w0 = sh.z[i][c0], w1 = sh.z[i][c0 + 1];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            acc[u][0] += rv[u] * w0;
            acc[u][1] += rv[u] * w1;
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c2 = c20 + u;
          if (c2 < K) {
            const double dd = sh.dsc[c2];
            const double sc = dd > 0.0 ? 1.0 / dd : 0.0;
            sh.gy[c2][c0] = acc[u][0] * sc;
            if (c0 + 1 < k) sh.gy[c2][c0 + 1] = acc[u][1] * sc;
          }
        }
      }
    }
    __syncthreads();
    // 7. new factors, streamed in place; then the new rank
    trunc_apply2(sh, U, V, m, n, K, k);
    if (tid == 0) *gptr<int32_t>(U.rankp) = k;
    __threadfence_block();
    __syncthreads();
    // work of this pass at the sizes it actually ran: the Grams (symmetric
    // halves) and their pivoted Cholesky, M = R S^T, the optional reduction
    // (M M^T and its stopped Cholesky), the Jacobi rotations executed (12 rx
    // flops per column pair and sweep), the small Tx / Ty products and
    // triangular solve, and the recombination of the new factors
    {
      const double dK = K, dm = m + n, drx = rx, dry = ry, djc = jc;
      double f = dm * dK * (dK + 1.0) + 2.0 * dK * dK * dK / 3.0 + 2.0 * drx * dry * dK;
      if (reduced) f += drx * (drx + 1.0) * dry + drx * djc * djc;
      f += 6.0 * drx * djc * (djc - 1.0) * sweeps;
      f += 2.0 * drx * dK * k + drx * drx * k + 2.0 * dm * dK * k;
      flops += f;
    }
    bytes += es * (double)(m + n) * (K + k);
  }
  // detail: passes, Jacobi sweeps, largest Cholesky ranks of the two sides
  put_cost(op, flops, bytes, (double)capped_any, (double)sh.k, (double)Kmax,
           passes * 1e9 + sweeps_all * 1e6 + rxmax * 1e3 + rymax);
}

// ---------------------------------------------------------------- solve updates
// T := V^T X (V: n x k panel, X: n x nrhs FP64, T: FP64 with ld >= k; with
// i2 = 1, T += V^T X), rows streamed in chunks of 64; each thread prefetches
// the next chunk into registers while the current one is multiplied.
#define LDS_MVT (2 * 64 * 65 * 8)
__device__ __forceinline__ void mvt_body(const Op& op) {
  char* const smem = hlu_lds;
  const PRef V = op.p[0], X = op.p[2], T = op.p[3];
  // the live rank k and right-hand-side count nr are read from device
  // memory; the loads are addressed by the stored widths, so they need not
  // wait for those reads, and k and nr only mask the chunks in LDS
  const int n = V.rows, k = pcols(V), nr = pcols(X);
  double (*sv)[65] = reinterpret_cast<double (*)[65]>(smem);
  double (*sx)[65] = reinterpret_cast<double (*)[65]>(smem + 64 * 65 * 8);
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  // T^T = X^T V on the matrix cores (the sixteen lanes of a result register
  // then hold consecutive rows of T): 16 x 16 tiles over (nrhs, k), tile
  // w + 4j to wavefront w; rows in chunks of 64 (one leaf: one round trip)
  const int nta = (k + 15) >> 4, ntile = nta * ((nr + 15) >> 4);
  v4d acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = (v4d){0.0, 0.0, 0.0, 0.0};
  double pv[16], px[16];
  const GView gv = gview(V), gx = gview(X);
  // loads only: lanes outside V or X read a clamped element and are zeroed
  // when the chunk is stored to LDS, so the prefetch stays in flight
  auto fetch = [&](int r0) {
    int ri[16], cv[16], cx[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int q = tid + NT * u, i = q & 63, j = q >> 6;
      ri[u] = min(r0 + i, n - 1);
      cv[u] = min(j, V.cols - 1);
      cx[u] = min(j, X.cols - 1);
    }
    gload(gv, ri, cv, pv);
    gload(gx, ri, cx, px);
  };
  const int nn = (V.cols > 0 && X.cols > 0) ? n : 0;
  if (nn > 0) fetch(0);
  for (int r0 = 0; r0 < nn; r0 += 64) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int q = tid + NT * u, i = q & 63, j = q >> 6;
      const bool in = r0 + i < n;
      sv[i][j] = (in && j < k) ? pv[u] : 0.0;
      sx[i][j] = (in && j < nr) ? px[u] : 0.0;
    }
    __syncthreads();
    if (r0 + 64 < nn) fetch(r0 + 64);
    // all 16 steps of the chunk, straight-line (rows beyond n are zero)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int tt = w + 4 * j;
      if (tt < ntile) {
        const int a0 = 16 * (tt % nta), b0 = 16 * (tt / nta);
#pragma unroll 4
        for (int q = 0; q < 16; ++q) {
          const int i = 4 * q + (l >> 4);
          acc[j] = mfma16x16x4(sx[i][b0 + (l & 15)], sv[i][a0 + (l & 15)], acc[j]);
        }
      }
    }
    __syncthreads();
  }
  HLU_G double* t = gptr<double>(T.ptr);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int tt = w + 4 * j;
    if (tt < ntile) {
      const int a0 = 16 * (tt % nta), b0 = 16 * (tt / nta);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = a0 + (l & 15), b = b0 + (l >> 4) + 4 * r;
        if (a < k && b < nr) {
          // i2 = 1: accumulate onto the partial product of the other rows
          const size_t o = a + (size_t)b * T.ld;
          t[o] = op.i2 == 1 ? t[o] + acc[j][r] : acc[j][r];
        }
      }
    }
  }
  const double es = V.dt == DT_F64 ? 8.0 : 4.0;
  put_cost(op, 2.0 * n * k * nr, es * n * k + 8.0 * n * nr + 8.0 * k * nr);
}

// Y += d0 * sum_t X_t Y_t over the terms of one leaf row cluster (Y: rows
// <= 64 x nrhs <= 64, FP64; X_t: rows x kk_t, kk_t = live columns <= 64,
// FP32 or FP64; Y_t: FP64, ld >= kk_t; all plain column-major, checked on
// the host).  The work items are the 16-column chunks of the terms, dealt to
// the four wavefronts in turn; a wavefront stages its chunk in its own LDS
// slice (no block barrier inside the loop) and lane r accumulates row r of
// its partial in registers.  The four partials are summed once at the end.
#define MVR_TMAX 256
#define MVR_STAGE (4 * (64 * 17 + 16 * 65) * 8)
#define MVR_W (MVR_STAGE + 2 * MVR_TMAX * 4 + MVR_TMAX * 80)   // fused leaf inverse
#define MVR_Y (MVR_W + 64 * 65 * 8)                             // its updated rows
#define LDS_MVROW (MVR_Y + 64 * 65 * 8)
static_assert(LDS_MVROW <= 160 * 1024, "row update LDS");
static_assert(sizeof(Term) == 80, "term records are staged as ten 8-byte words");
__device__ __forceinline__ void mvrow_body(const Op& op) {
  char* const smem = hlu_lds;
  const PRef Y = op.p[3];
  // nr (the live right-hand sides) and a low-rank term's live width are read
  // from device memory; loads are addressed by the static capacities (Y.cols,
  // the term's cols) so they need not wait for those reads, and the live
  // counts only mask products and stores
  const int nt = min(op.i1, MVR_TMAX), rows = Y.rows, nr = pcols(Y), ncap = Y.cols;
  const double d0 = op.d0;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  double (*sa)[17] = reinterpret_cast<double (*)[17]>(smem + w * (64 * 17 + 16 * 65) * 8);
  double (*sb)[65] = reinterpret_cast<double (*)[65]>(smem + w * (64 * 17 + 16 * 65) * 8 +
                                                      64 * 17 * 8);
  int* kk = reinterpret_cast<int*>(smem + MVR_STAGE);
  int* first = kk + MVR_TMAX;   // first work item of each term
  // the term records, staged once (every work item reads its term's
  // pointers and strides from here instead of global memory)
  Term* st = reinterpret_cast<Term*>(smem + MVR_STAGE + 2 * MVR_TMAX * 4);
  // fused leaf inverse (i2 = 1): W staged beside the tables, the updated
  // rows of every right-hand-side group collected in a region of their own
  // (the staging area is reused by the next group), then p3 := W p3
  const bool fused = op.i2 == 1;
  double (*sw)[65] = reinterpret_cast<double (*)[65]>(smem + MVR_W);
  double (*sy)[65] = reinterpret_cast<double (*)[65]>(smem + MVR_Y);
  // W's loads are issued here and stay in flight through the term products;
  // it reaches LDS only before the first reduction barrier
  double wv[16];
  if (fused) {
    const PRef W = op.p[0];
    const HLU_G double* gw = gptr<const double>(W.ptr);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + NT * u, i = e & 63, j = e >> 6;
      wv[u] = (i < rows && j < rows) ? gw[i + (size_t)j * W.ld] : 0.0;
    }
  }
  // one term carried in the op itself (p1 its factor, p2 its operand): read
  // from the descriptor, with no staging and no barrier before the loads
  const bool inl = op.i0 < 0;
  int kk0 = 0;
  if (inl) {
    kk0 = pcols(op.p[1]);
  } else {
    const HLU_G uint64_t* src = gptr<const uint64_t>(op.p[2].ptr) + (size_t)op.i0 * 10;
    uint64_t* dst = reinterpret_cast<uint64_t*>(st);
    for (int e = tid; e < nt * 10; e += NT) dst[e] = src[e];
    __syncthreads();
    for (int t = tid; t < nt; t += NT) kk[t] = pcols(st[t].X);
    __syncthreads();
    if (tid == 0) {
      int acc = 0;
      for (int t = 0; t < nt; ++t) {
        first[t] = acc;
        acc += (kk[t] + 15) >> 4;
      }
    }
    __syncthreads();
  }
  const int nitems = inl ? (op.p[1].cols + 15) >> 4
                         : nt > 0 ? first[nt - 1] + ((kk[nt - 1] + 15) >> 4) : 0;
  // item -> (term, first column): a short scan over the terms
  auto locate = [&](int item, int& t, int& c0) {
    t = 0;
    while (t + 1 < nt && first[t + 1] <= item) ++t;
    c0 = (item - first[t]) * 16;
  };
  // the four wavefronts' partials side by side (staging area, free after the terms)
  double (*part)[64][33] = reinterpret_cast<double (*)[64][33]>(smem);
  // right-hand sides in groups of 32 (one group when nrhs <= 32)
  // chunk `item` (16 columns of one term) of the A panel (lane = row) and of
  // the B panel (lane = right-hand side h0 + lane) into registers
  // Lanes beyond the rows or right-hand sides and columns beyond kc read a
  // clamped element: their products land only in outputs that are never
  // stored, so nothing is zeroed and all 32 loads are issued together.
  auto fetch = [&](int item, int h0, int nh, double (&ra)[16], double (&rb)[16], int& kc) {
    int t = 0, c0 = item * 16;
    if (!inl) locate(item, t, c0);
    const PRef& tX = inl ? op.p[1] : st[t].X;
    const PRef& tY = inl ? op.p[2] : st[t].Y;
    // columns clamped to the stored width (inline) or the live one
    const int kcs = min(16, (inl ? tX.cols : kk[t]) - c0);
    int ri[16], cj[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      ri[u] = min(lane, rows - 1);
      cj[u] = c0 + min(u, kcs - 1);
    }
    kc = min(kcs, (inl ? kk0 : kk[t]) - c0);
    gload(gview(tX), ri, cj, ra);
    const HLU_G double* pb =
        gptr<const double>(tY.ptr) + (size_t)(h0 + min(lane, nh - 1)) * tY.ld;
#pragma unroll
    for (int u = 0; u < 16; ++u) rb[u] = pb[cj[u]];
  };
  for (int h0 = 0; h0 < ncap; h0 += 32) {
    const int nh = min(32, nr - h0), nhs = min(32, ncap - h0);   // live, stored
    // the old values of the rows, eight right-hand sides per wavefront (the
    // ones it finishes below), in flight while the terms are multiplied;
    // lanes beyond the rows or right-hand sides read a clamped element
    double yv[8];
    {
      const HLU_G double* y = gptr<const double>(Y.ptr) + min(lane, rows - 1) + (size_t)h0 * Y.ld;
#pragma unroll
      for (int v = 0; v < 8; ++v) yv[v] = y[(size_t)min(8 * w + v, nhs - 1) * Y.ld];
    }
    // this wavefront's partial (64 rows x 32 right-hand sides) as eight
    // 16 x 16 matrix-core tiles: row block ti, column block tj in acc[2 ti + tj]
    v4d acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = (v4d){0.0, 0.0, 0.0, 0.0};
    for (int item = w; item < nitems; item += 4) {
      double ra[16], rb[16];
      int kc;
      fetch(item, h0, nhs, ra, rb, kc);
      // the slices were last read by this wavefront's previous chunk (program order)
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        sa[lane][u] = ra[u];
        sb[u][lane] = rb[u];
      }
      // partial += A B over the chunk's 16 columns, four per step (columns
      // at or beyond kc hold clamped copies and enter as zeros)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = 4 * q + (lane >> 4);
        const bool in = c < kc;
        double bq[2];
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
          const double v = sb[c][16 * tj + (lane & 15)];
          bq[tj] = in ? v : 0.0;
        }
#pragma unroll
        for (int ti = 0; ti < 4; ++ti) {
          const double av = sa[16 * ti + (lane & 15)][c];
          const double aq = in ? av : 0.0;
#pragma unroll
          for (int tj = 0; tj < 2; ++tj) acc[2 * ti + tj] = mfma16x16x4(aq, bq[tj], acc[2 * ti + tj]);
        }
      }
    }
    // the four partials side by side in the (now free) staging area; then
    // wavefront w sums right-hand sides 8w .. 8w + 7 of all four and
    // updates them (in a fixed order: partial 0, 1, 2, 3)
    if (fused && h0 == 0) {
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = tid + NT * u, i = e & 63, j = e >> 6;
        sw[i][j] = wv[u];
      }
    }
    __syncthreads();
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          part[w][16 * ti + (lane >> 4) + 4 * r][16 * tj + (lane & 15)] = acc[2 * ti + tj][r];
    __syncthreads();
    {
      // fused: every row and column of the group goes to sy, zero outside
      // the rows and the live right-hand sides, so that the product with W
      // below reads sy without selects
      HLU_G double* y = gptr<double>(Y.ptr) + min(lane, rows - 1) + (size_t)h0 * Y.ld;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int c = 8 * w + v;
        const bool ok = lane < rows && c < nh;
        const double sum = ((part[0][lane][c] + part[1][lane][c]) + part[2][lane][c]) +
                           part[3][lane][c];
        const double val = yv[v] + d0 * sum;
        if (fused) sy[lane][h0 + c] = ok ? val : 0.0;
        else if (ok) y[(size_t)c * Y.ld] = val;
      }
    }
    __syncthreads();
  }
  if (fused) {
    // p3 := W (updated rows) on the matrix cores, taken transposed
    // ((W S)^T = S^T W^T) so that the sixteen lanes of a result register
    // hold consecutive rows; wavefront w takes rows 16w .. 16w + 15 and the
    // column tiles two at a time (one read of W per step, two independent
    // accumulation chains)
    const int ntj = (nr + 15) >> 4;
    HLU_G double* gy = gptr<double>(Y.ptr);
    const int i0 = 16 * w;
    if (i0 < rows) {
      for (int jt = 0; jt < ntj; jt += 2) {
        const int j0 = 16 * jt, j1 = j0 + 16;
        const bool two = jt + 1 < ntj;
        v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
        // all 16 steps, straight-line: W and sy are zero beyond the rows,
        // and sy beyond the live right-hand sides (a second tile past the
        // last one reads zeros)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int k = 4 * q + (lane >> 4);
          const double b = sw[i0 + (lane & 15)][k];
          acc0 = mfma16x16x4(sy[k][j0 + (lane & 15)], b, acc0);
          acc1 = mfma16x16x4(sy[k][j1 + (lane & 15)], b, acc1);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + (lane & 15), j = j0 + (lane >> 4) + 4 * r;
          if (i < rows && j < nr) gy[i + (size_t)j * Y.ld] = acc0[r];
          if (two && i < rows && j + 16 < nr) gy[i + (size_t)(j + 16) * Y.ld] = acc1[r];
        }
      }
    }
  }
  if (tid == 0 && op.cost) {
    double fl = fused ? 2.0 * rows * rows * nr : 0.0;
    double by = 16.0 * rows * nr + (fused ? 8.0 * rows * rows : 0.0);
    for (int t = 0; t < nt; ++t) {
      const PRef A = inl ? op.p[1] : st[t].X;
      const int k = inl ? kk0 : kk[t];
      fl += 2.0 * rows * k * nr;
      by += (A.dt == DT_F64 ? 8.0 : 4.0) * rows * k + 8.0 * k * nr;
    }
    put_cost(op, fl, by);
  }
}

// ---------------------------------------------------------------- matvec
// T_b = V_b^T X[c0:c0+n, :] for every low-rank block b of the matvec copy:
// rows in chunks of 32, the next chunk loading while the current one is
// multiplied; T^T = X^T V on the matrix cores (16 x 16 tiles over the
// right-hand sides and the rank, tile w + 4j to wavefront w).
__global__ void __launch_bounds__(NT) k_mv_t(const MvLR* __restrict__ lr, const double* X,
                                             int ldx, int nrhs) {
  const MvLR e = lr[blockIdx.x];
  if (e.k == 0 || e.n <= 0) return;
  const HLU_G double* V = gptr<const double>(e.V);
  const HLU_G double* gx = gptr<const double>((uint64_t)X);
  HLU_G double* T = gptr<double>(e.T);
  __shared__ double sv[32][65];
  __shared__ double sx[32][65];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  for (int k0 = 0; k0 < e.k; k0 += 64) {
    const int kk = min(64, e.k - k0);
    for (int c0 = 0; c0 < nrhs; c0 += 64) {
      const int wc = min(64, nrhs - c0);
      const int nta = (kk + 15) >> 4, ntile = nta * ((wc + 15) >> 4);
      v4d acc[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] = (v4d){0.0, 0.0, 0.0, 0.0};
      double pv[8], px[8];
      auto fetch = [&](int r0) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int q = tid + NT * u, i = q & 31, j = q >> 5;
          const int row = min(r0 + i, e.n - 1);
          pv[u] = V[(size_t)row + (size_t)(k0 + min(j, kk - 1)) * e.n];
          px[u] = gx[(size_t)(e.c0 + row) + (size_t)(c0 + min(j, wc - 1)) * ldx];
        }
      };
      fetch(0);
      for (int r0 = 0; r0 < e.n; r0 += 32) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int q = tid + NT * u, i = q & 31, j = q >> 5;
          const bool in = r0 + i < e.n;
          sv[i][j] = (in && j < kk) ? pv[u] : 0.0;
          sx[i][j] = (in && j < wc) ? px[u] : 0.0;
        }
        __syncthreads();
        if (r0 + 32 < e.n) fetch(r0 + 32);
        const int nq = (min(32, e.n - r0) + 3) >> 2;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int tt = w + 4 * j;
          if (tt < ntile) {
            const int a0 = 16 * (tt % nta), b0 = 16 * (tt / nta);
            for (int q = 0; q < nq; ++q) {
              const int i = 4 * q + (l >> 4);
              acc[j] = mfma16x16x4(sx[i][b0 + (l & 15)], sv[i][a0 + (l & 15)], acc[j]);
            }
          }
        }
        __syncthreads();
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int tt = w + 4 * j;
        if (tt < ntile) {
          const int a0 = 16 * (tt % nta), b0 = 16 * (tt / nta);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int a = a0 + (l & 15), b = b0 + (l >> 4) + 4 * r;
            if (a < kk && b < wc) T[(size_t)(k0 + a) + (size_t)(c0 + b) * e.kcap] = acc[j][r];
          }
        }
      }
    }
  }
}

// y[rows of leaf] = beta * b + alpha * sum over the leaf row's blocks (F X or
// U T): (0, 1) gives y = A X, (1, -1) the residual b - A X.  Lane i holds row
// i for 32 right-hand sides at a time and the four wavefronts take alternate
// columns of every block, so each matrix entry is read once; the slices of X
// (or T) for 64 columns at a time are staged in LDS and read as broadcasts,
// and the four partial sums meet in LDS at the end.
__global__ void __launch_bounds__(NT) k_mv_rows(const MvRow* __restrict__ rows,
                                                const MvTerm* __restrict__ terms,
                                                const double* X, int ldx, const double* B,
                                                double beta, double alpha, double* Yo,
                                                int nrhs) {
  const MvRow r = rows[blockIdx.x];
  __shared__ __align__(16) double sx[64][34];
  __shared__ double red[2][64][33];
  const int tid = threadIdx.x, i = tid & 63, g = tid >> 6;
  if (r.rows <= 0) return;
  const int ir = min(i, r.rows - 1);
  const HLU_G double* gx = gptr<const double>((uint64_t)X);
  for (int h0 = 0; h0 < nrhs; h0 += 32) {
    const int nh = min(32, nrhs - h0);
    double acc[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) acc[j] = 0.0;
    for (int q = 0; q < r.nt; ++q) {
      const MvTerm t = terms[r.t0 + q];
      const HLU_G double* A = gptr<const double>(t.A) + t.roff + ir;
      for (int cc = 0; cc < t.ncol; cc += 64) {
        const int nc = min(64, t.ncol - cc);
        {
          // sx[c][j] = X[c0 + cc + c][h0 + j] (dense) or T[cc + c][h0 + j]
          // (low rank); lanes beyond nc or nh read a clamped element that no
          // product uses
          const int cl = cc + min(i, nc - 1);
          double v[8];
          if (t.T == 0) {
#pragma unroll
            for (int u = 0; u < 8; ++u)
              v[u] = gx[(size_t)(t.c0 + cl) + (size_t)(h0 + min(g + 4 * u, nh - 1)) * ldx];
          } else {
            const HLU_G double* T = gptr<const double>(t.T);
#pragma unroll
            for (int u = 0; u < 8; ++u)
              v[u] = T[(size_t)cl + (size_t)(h0 + min(g + 4 * u, nh - 1)) * t.c0];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) sx[i][g + 4 * u] = v[u];
        }
        __syncthreads();
        for (int c = g; c < nc; c += 16) {
          double a[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) a[u] = A[(size_t)(cc + min(c + 4 * u, nc - 1)) * t.lda];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (c + 4 * u < nc) {
              const double* xr = &sx[c + 4 * u][0];
              double xv[32];
#pragma unroll
              for (int j = 0; j < 32; ++j) xv[j] = xr[j];
#pragma unroll
              for (int j = 0; j < 32; ++j) acc[j] += a[u] * xv[j];
            }
          }
        }
        __syncthreads();
      }
    }
    if (g >= 2) {
#pragma unroll
      for (int j = 0; j < 32; ++j) red[g - 2][i][j] = acc[j];
    }
    __syncthreads();
    if (g < 2) {
#pragma unroll
      for (int j = 0; j < 32; ++j) acc[j] += red[g][i][j];
    }
    __syncthreads();
    if (g == 1) {
#pragma unroll
      for (int j = 0; j < 32; ++j) red[0][i][j] = acc[j];
    }
    __syncthreads();
    if (g == 0 && i < r.rows) {
#pragma unroll
      for (int j = 0; j < 32; ++j) {
        if (j < nh) {
          const size_t o = (size_t)(r.r0 + i) + (size_t)(h0 + j) * ldx;
          Yo[o] = beta * (B ? B[o] : 0.0) + alpha * (acc[j] + red[0][i][j]);
        }
      }
    }
    __syncthreads();
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

// X[:, j] += D[:, j] for the columns with active[j] != 0 (refinement keeps
// converged columns as they are)
__global__ void k_axpy_masked(double* X, const double* D, int ld, int n, int nrhs,
                              const int32_t* active) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * nrhs) return;
  int p = (int)(e % n), j = (int)(e / n);
  if (active[j]) X[p + (size_t)j * ld] += D[p + (size_t)j * ld];
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

__global__ void k_keep_flag(const int32_t* src, int32_t* dst) {
  if (threadIdx.x == 0 && *src != 0 && *dst == 0) *dst = *src;
}
__global__ void k_set_int(int32_t* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// ---------------------------------------------------------------- leaf inverses
// From the factored leaf (b x b, L unit lower and U in place) and its
// interchanges: W = L^{-1} P (so that W y = L^{-1} P y) and U^{-1}, both
// b x b FP64 with leading dimension b.  Column k of L^{-1} is the forward
// substitution of e_k (one thread per column, threads 0-63), column k of
// U^{-1} the backward substitution of e_k (threads 64-127).  The solve then
// applies each leaf step as one small dense product.
#define LDS_TRINV (3 * 64 * 65 * 8 + 64 * 4)
static_assert(LDS_TRINV <= sizeof(TruncShared), "the factor executor's LDS holds the inverses");
__device__ void d_trinv(const Op& op) {
  char* const smem = hlu_lds;
  const PRef A = op.p[0], W = op.p[2], Ui = op.p[3];
  const int b = A.rows;
  double (*l)[65] = reinterpret_cast<double (*)[65]>(smem);
  double (*x)[65] = reinterpret_cast<double (*)[65]>(smem + 64 * 65 * 8);
  double (*y)[65] = reinterpret_cast<double (*)[65]>(smem + 2 * 64 * 65 * 8);
  int* pm = reinterpret_cast<int*>(smem + 3 * 64 * 65 * 8);
  const int tid = threadIdx.x;
  {
    const HLU_G double* g = gptr<const double>(A.ptr);
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + NT * u, i = e & 63, j = e >> 6;
      v[u] = (i < b && j < b) ? g[i + (size_t)j * A.ld] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + NT * u, i = e & 63, j = e >> 6;
      l[i][j] = v[u];
    }
  }
  if (tid < 64) {
    // row permutation of the interchanges applied in order: lane i holds
    // the source row of position i
    const HLU_G int32_t* piv = gptr<const int32_t>(op.p[1].ptr);
    const int pk = tid < b ? piv[tid] : tid;
    int pr = tid;
    for (int k = 0; k < b; ++k) {
      const int p = __builtin_amdgcn_readlane(pk, k);
      const int vk = __builtin_amdgcn_readlane(pr, k), vp = __builtin_amdgcn_readlane(pr, p);
      pr = tid == k ? vp : (tid == p ? vk : pr);
    }
    pm[tid] = pr;
  }
  __syncthreads();
  if (tid < 64) {
    const int k = tid;
    if (k < b) {
      for (int i = 0; i < b; ++i) {
        double v = i == k ? 1.0 : 0.0;
        if (i > k) {
          double sacc = 0.0;
          for (int m = k; m < i; ++m) sacc += l[i][m] * x[m][k];
          v = -sacc;
        }
        x[i][k] = v;
      }
    }
  } else if (tid < 128) {
    const int k = tid - 64;
    if (k < b) {
      for (int i = b - 1; i >= 0; --i) {
        double v = 0.0;
        if (i <= k) {
          double sacc = i == k ? 1.0 : 0.0;
          for (int m = i + 1; m <= k; ++m) sacc -= l[i][m] * y[m][k];
          v = sacc / l[i][i];
        }
        y[i][k] = v;
      }
    }
  }
  __syncthreads();
  HLU_G double* w = gptr<double>(W.ptr);
  HLU_G double* u = gptr<double>(Ui.ptr);
  for (int e = tid; e < b * b; e += NT) {
    const int i = e % b, k = e / b;
    w[i + (size_t)pm[k] * b] = x[i][k];
    u[i + (size_t)k * b] = y[i][k];
  }
  put_cost(op, 2.0 * b * b * b / 3.0, 24.0 * b * b);
}

// p1 := W p1 for a leaf inverse W (b x b) and the b x nrhs panel p1 (FP64):
// both staged in LDS, 16 x 16 threads with 4 x 4 outputs each.
#define LDS_INVAPPLY (2 * 64 * 65 * 8)
__device__ __forceinline__ void invapply_body(const Op& op) {
  char* const smem = hlu_lds;
  const PRef Wr = op.p[0], Y = op.p[1];
  const int b = Wr.rows, nr = pcols(Y);
  double (*w)[65] = reinterpret_cast<double (*)[65]>(smem);
  double (*y)[65] = reinterpret_cast<double (*)[65]>(smem + 64 * 65 * 8);
  const int tid = threadIdx.x;
  const HLU_G double* gw = gptr<const double>(Wr.ptr);
  HLU_G double* gy = gptr<double>(Y.ptr);
  {
    double v[16], q[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + NT * u, i = e & 63, j = e >> 6;
      v[u] = (i < b && j < b) ? gw[i + (size_t)j * Wr.ld] : 0.0;
      q[u] = (i < b && j < nr) ? gy[i + (size_t)j * Y.ld] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + NT * u, i = e & 63, j = e >> 6;
      w[i][j] = v[u];
      y[i][j] = q[u];
    }
  }
  __syncthreads();
  const int ti = tid % 16, tj = tid / 16;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int k = 0; k < b; ++k) {
    double av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) av[u] = w[ti + 16 * u][k];
#pragma unroll
    for (int v = 0; v < 4; ++v) bv[v] = y[k][tj + 16 * v];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] += av[u] * bv[v];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = ti + 16 * u, j = tj + 16 * v;
      if (i < b && j < nr) gy[i + (size_t)j * Y.ld] = acc[u][v];
    }
  put_cost(op, 2.0 * b * b * nr, 8.0 * b * b + 16.0 * b * nr);
}

// Out-of-line entries of the leaf solve, panel product, dense update, zeroing
// and H-matvec update bodies for the wave kernel.  The dataflow executors
// take the bodies inline, so no registers are saved across a call.
__device__ __noinline__ void d_trsm(const Op& op) { trsm_body(op); }
__device__ __noinline__ void d_pgemm(const Op& op) { pgemm_body(op); }
__device__ __noinline__ void d_addd(const Op& op) { addd_body(op); }
__device__ __noinline__ void d_zero(const Op& op) { zero_body(op); }
__device__ __noinline__ void d_mvt(const Op& op) { mvt_body(op); }
__device__ __noinline__ void d_mvrow(const Op& op) { mvrow_body(op); }
__device__ __noinline__ void d_invapply(const Op& op) { invapply_body(op); }

// ---------------------------------------------------------------- launchers
// One workgroup per descriptor; the descriptors of a launch may mix op
// types (one launch per wave of the schedule).  Each op type carves its
// tiles out of the same dynamic LDS buffer, so a launch requests the
// largest footprint among the types it contains.
__device__ __forceinline__ void run_op_body(const Op& op) {
  switch (op.type) {
    case OP_GETRF: d_getrf(op); break;
    case OP_TRSM_L:
    case OP_TRSM_UT:
    case OP_TRSM_U: d_trsm(op); break;
    case OP_PGEMM: d_pgemm(op); break;
    case OP_TRUNC: d_trunc(op); break;
    case OP_ADDD: d_addd(op); break;
    case OP_ZERO: d_zero(op); break;
    case OP_MVT: d_mvt(op); break;
    case OP_MVROW: d_mvrow(op); break;
    case OP_TRINV: d_trinv(op); break;
    case OP_INVAPPLY: d_invapply(op); break;
    default: break;
  }
}
__device__ __forceinline__ void run_op(const Op& op) {
  const long long t0 = wall_clock64();
  run_op_body(op);
  put_start(op, t0);
}

__global__ void __launch_bounds__(NT) k_wave(const Op* __restrict__ ops) {
  run_op(ops[blockIdx.x]);
}

// ---------------------------------------------------------------- dataflow
// Persistent executor of a whole schedule (factor or solve): the device analogue of
// running nested tasks with weak dependencies and early release (Sec. 5.2)
// -- an op starts as soon as its own predecessors have finished, across
// recursion levels, instead of waiting for a whole wave.
//   ctrl[0]: next queue slot to take, ctrl[1]: next slot to fill,
//   ctrl[2]: error flag (1: a wait exceeded the time limit, 2: queue
//   overflow, 3: an op type this executor does not run).
// Every op is pushed exactly once (when its last predecessor finishes), so
// the queue has one slot per op; a workgroup that takes a slot >= n exits.
// Waits are bounded by `timeout` ticks of the constant-rate wall clock, after
// which the error flag is raised and every waiting workgroup exits.
// part owning global op index g (the last part whose base is <= g)
__device__ __forceinline__ int df_part(const DfPart* parts, int np, int g) {
  int lo = 0, hi = np - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (parts[mid].base <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void k_df_reset(const DfPart* parts, int np, int* queue, const int* ready0, int nready,
                           int n, int* ctrl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const DfPart& pt = parts[df_part(parts, np, i)];
    const int l = i - pt.base;
    reinterpret_cast<int*>(pt.indeg)[l] = reinterpret_cast<const int*>(pt.indeg0)[l];
    queue[i] = i < nready ? ready0[i] : -1;
  }
  if (i == 0) {
    ctrl[0] = 0;        // low ring: next ticket
    ctrl[1] = nready;   // low ring: next free slot
    ctrl[2] = 0;        // error flag
    ctrl[3] = 0;        // high ring: next ticket
    ctrl[4] = 0;        // high ring: next free slot
    ctrl[6] = 0;        // ops finished
  }
}

// Op types each executor instantiation runs: the factor schedule's and the
// solve schedule's (the host validates every schedule against its mask; an op
// outside it raises error 3).
constexpr unsigned DF_FACTOR_TYPES = (1u << OP_GETRF) | (1u << OP_TRSM_L) | (1u << OP_TRSM_UT) |
                                     (1u << OP_TRSM_U) | (1u << OP_PGEMM) | (1u << OP_TRUNC) |
                                     (1u << OP_ADDD) | (1u << OP_ZERO) | (1u << OP_TRINV);
constexpr unsigned DF_SOLVE_TYPES = (1u << OP_MVT) | (1u << OP_MVROW) | (1u << OP_INVAPPLY);

template <unsigned MASK>
__device__ __forceinline__ bool run_op_masked_body(const Op& op, int tune) {
  switch (op.type) {
    case OP_GETRF: if constexpr ((MASK >> OP_GETRF) & 1) { d_getrf(op); return true; } break;
    case OP_TRSM_L:
    case OP_TRSM_UT:
    case OP_TRSM_U:
      if constexpr (MASK & ((1u << OP_TRSM_L) | (1u << OP_TRSM_UT) | (1u << OP_TRSM_U))) {
        trsm_body(op);
        return true;
      }
      break;
    case OP_PGEMM: if constexpr ((MASK >> OP_PGEMM) & 1) { pgemm_body(op); return true; } break;
    case OP_TRUNC: if constexpr ((MASK >> OP_TRUNC) & 1) { d_trunc(op, tune); return true; } break;
    case OP_ADDD: if constexpr ((MASK >> OP_ADDD) & 1) { addd_body(op); return true; } break;
    case OP_ZERO: if constexpr ((MASK >> OP_ZERO) & 1) { zero_body(op); return true; } break;
    case OP_MVT:
      if constexpr ((MASK >> OP_MVT) & 1) {
        mvt_body(op);
        return true;
      }
      break;
    case OP_MVROW:
      if constexpr ((MASK >> OP_MVROW) & 1) {
        mvrow_body(op);
        return true;
      }
      break;
    case OP_TRINV: if constexpr ((MASK >> OP_TRINV) & 1) { d_trinv(op); return true; } break;
    case OP_INVAPPLY:
      if constexpr ((MASK >> OP_INVAPPLY) & 1) {
        invapply_body(op);
        return true;
      }
      break;
    default: break;
  }
  return false;
}
template <unsigned MASK>
__device__ __forceinline__ bool run_op_masked(const Op& op, int tune) {
  const long long t0 = wall_clock64();
  const bool ok = run_op_masked_body<MASK>(op, tune);
  put_start(op, t0);
  return ok;
}

// The ready ops sit in two FIFO rings of one queue array: the low ring
// (slots [0, n - nhigh)) and the high ring (slots [n - nhigh, n)) for the ops
// flagged as near-critical (bit 30 of their initial in-degree).  Workgroups
// 0 .. nhw - 1 serve the high ring, the others the low ring, each with the
// same protocol: take a ticket, wait for the op pushed into that slot.
// The initially ready ops are never flagged.  With nhw == 0 the flags are
// ignored (one ring).  A workgroup whose decrements make successors ready
// keeps the first of them (lowest position in its successor list, among the
// first NT) and runs it next without going through a ring; the others are
// pushed.  Kept ops leave slots of the rings unfilled, so a waiting
// workgroup also leaves once all n ops have finished (a counter).
// an op descriptor as 32-bit words (staged in LDS by the dataflow executor)
constexpr int DF_OPW = (int)(sizeof(Op) / 4);
static_assert(sizeof(Op) % 4 == 0 && DF_OPW + 2 <= 64, "descriptor staging by the first wavefront");
__device__ __forceinline__ int* s_desc_w(Op& o) { return reinterpret_cast<int*>(&o); }

template <unsigned MASK>
__device__ __forceinline__ void df_run(const DfPart* __restrict__ parts, int np, int* queue,
                                       int* ctrl, int n, int nhigh, int nhw, long long timeout) {
  __shared__ int s_op;
  __shared__ int s_keep;
  __shared__ int s_next;
  __shared__ Op s_desc;       // the running op's descriptor
  __shared__ int s_soff[2];   // and its successor range
  const int tid = threadIdx.x;
  if (nhw <= 0) nhigh = 0;
  const int nlow = n - nhigh;
  const bool hw = (int)blockIdx.x < nhw;
  int* const head = hw ? &ctrl[3] : &ctrl[0];
  int* const ring = hw ? queue + nlow : queue;
  const int cnt = hw ? nhigh : nlow;
  int* const finished = &ctrl[6];
  int next = -1;            // successor kept by the last op (thread 0)
  bool have = false;        // s_desc and s_soff already hold that op's (uniform)
  for (;;) {
    if (tid == 0) {
      int v = next;
      next = -1;
      if (v >= 0) {
        // made ready by this workgroup's own decrement, whose wavefront
        // acquired; once more here for the wavefront that reads the inputs
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      } else {
        const int s = __hip_atomic_fetch_add(head, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (s < cnt) {
          const long long t0 = (long long)wall_clock64();
          // spin with relaxed loads: an acquire per iteration would
          // invalidate this chiplet's L2 under the ops running beside it
          for (int it = 1;; ++it) {
            v = __hip_atomic_load(&ring[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (v >= 0) {
              // pairs with the release store that pushed v: the op's inputs
              // (every predecessor's writes) are visible from here on
              __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
              break;
            }
            if ((it & 31) == 0) {
              if (__hip_atomic_load(finished, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= n)
                break;   // every op has run: this slot stays empty
              if (__hip_atomic_load(&ctrl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
              if ((long long)wall_clock64() - t0 > timeout) {
                __hip_atomic_store(&ctrl[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
              }
            }
            __builtin_amdgcn_s_sleep(2);
          }
        }
      }
      s_op = v;
    }
    __syncthreads();
    const int g = s_op;
    if (g < 0) break;
    const DfPart& pt = parts[np == 1 ? 0 : df_part(parts, np, g)];
    const int idx = g - pt.base;
    const HLU_G int* succ_off = gptr<const int>(pt.succ_off);
    const HLU_G int* succ = gptr<const int>(pt.succ);
    const HLU_G int* opw = gptr<const int>(pt.ops);
    // the descriptor and successor range go to LDS in one round trip (a
    // kept op's were fetched while its predecessor's fence and decrements ran)
    if (!have) {
      if (tid < DF_OPW) s_desc_w(s_desc)[tid] = opw[(size_t)idx * DF_OPW + tid];
      else if (tid < DF_OPW + 2) s_soff[tid - DF_OPW] = succ_off[idx + tid - DF_OPW];
      __syncthreads();
    }
    // the successor list is static: it is read as the op starts and arrives
    // while the op runs, so only the decrements follow the op
    const int e0 = s_soff[0], e1 = s_soff[1];
    const int t_first = e0 + tid < e1 ? succ[e0 + tid] : -1;
    if (!run_op_masked<MASK>(s_desc, pt.tune) && tid == 0)
      __hip_atomic_store(&ctrl[2], 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // one release fence (first wavefront, after the barrier that completed
    // every wavefront's stores) publishes the op's writes; then all threads
    // decrement the successors' in-degrees at once (relaxed), so an op with
    // many successors pays one atomic round trip, not one per successor.
    // A thread that brings a successor to zero acquires (its decrement read
    // the others' through the chain of read-modify-writes, so their fences
    // synchronise with it) and pushes the successor with a release store
    // into the ring its flag names; each wavefront reserves the slots of its
    // pushes with one atomic per ring.  The lowest ready position among the
    // first NT successors is not pushed: this workgroup runs it next.
    __syncthreads();
    // the first successor is the one kept whenever it becomes ready: its
    // descriptor and successor range are fetched now (first wavefront,
    // thread 0's candidate), under the fence and the decrements
    int pre = 0;
    const int c = __builtin_amdgcn_readfirstlane(t_first);
    if (tid < DF_OPW + 2 && c >= 0)
      pre = tid < DF_OPW ? opw[(size_t)c * DF_OPW + tid] : succ_off[c + tid - DF_OPW];
    if (tid < 64) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (tid == 0) s_keep = 0x7fffffff;
    __syncthreads();
    {
      HLU_G int* indeg = gptr<int>(pt.indeg);
      const int lane = tid & 63;
      for (int eb = e0; eb < e1; eb += NT) {
        const int e = eb + tid;
        int t = -1;
        bool ready = false, hi = false;
        if (e < e1) {
          t = eb == e0 ? t_first : succ[e];
          const int old = __hip_atomic_fetch_add(&indeg[t], -1, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
          ready = (old & 0x3fffffff) == 1;
          hi = nhigh > 0 && ((old >> 30) & 1);
        }
        const unsigned long long mr = __ballot(ready);
        bool keep = false;
        if (eb == e0) {
          // the lowest ready position of the first chunk is kept
          if (mr && lane == __ffsll((long long)mr) - 1) atomicMin(&s_keep, e - e0);
          __syncthreads();
          keep = ready && e - e0 == s_keep;
          if (keep) s_next = pt.base + t;   // read by thread 0 after the barrier below
        }
        const unsigned long long mlo = __ballot(ready && !keep && !hi);
        const unsigned long long mhi = __ballot(ready && !keep && hi);
        if (mr) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
#pragma unroll
          for (int r = 0; r < 2; ++r) {
            const unsigned long long mask = r ? mhi : mlo;
            if (!mask) continue;
            const int leader = __ffsll((long long)mask) - 1;
            int slot0 = 0;
            if (lane == leader)
              slot0 = __hip_atomic_fetch_add(r ? &ctrl[4] : &ctrl[1], __popcll(mask),
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            slot0 = __shfl(slot0, leader);
            if ((mask >> lane) & 1ull) {
              const int slot = slot0 + __popcll(mask & ((1ull << lane) - 1ull));
              if (slot < (r ? nhigh : nlow))
                __hip_atomic_store(&queue[(r ? nlow : 0) + slot], pt.base + t, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
              else
                __hip_atomic_store(&ctrl[2], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
          }
        }
      }
    }
    __syncthreads();
    // position 0 kept: that is c, whose descriptor is in flight above (the
    // next iteration's first barrier orders these writes before its reads)
    have = s_keep == 0;
    if (have && tid < DF_OPW + 2) {
      if (tid < DF_OPW) s_desc_w(s_desc)[tid] = pre;
      else s_soff[tid - DF_OPW] = pre;
    }
    if (tid == 0) {
      if (s_keep != 0x7fffffff) next = s_next;
      __hip_atomic_fetch_add(finished, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

__global__ void __launch_bounds__(NT) k_df_factor(const DfPart* __restrict__ parts, int np,
                                                  int* queue, int* ctrl, int n, int nhigh,
                                                  int nhw, long long timeout) {
  df_run<DF_FACTOR_TYPES>(parts, np, queue, ctrl, n, nhigh, nhw, timeout);
}
__global__ void __launch_bounds__(NT) k_df_solve(const DfPart* __restrict__ parts, int np,
                                                 int* queue, int* ctrl, int n, int nhigh,
                                                 int nhw, long long timeout) {
  df_run<DF_SOLVE_TYPES>(parts, np, queue, ctrl, n, nhigh, nhw, timeout);
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
    case OP_MVT: return LDS_MVT;
    case OP_MVROW: return LDS_MVROW;
    case OP_TRINV: return LDS_TRINV;
    case OP_INVAPPLY: return LDS_INVAPPLY;
    default: return 0;
  }
}

// the largest dynamic LDS footprint of any op type (the wave kernel's limit)
static size_t max_lds_bytes() {
  size_t mx = 0;
  for (int t = 0; t < OP_NTYPES; ++t) mx = std::max(mx, lds_bytes(t));
  return mx;
}

static hipError_t launch_wave(const Op* ops, int count, size_t lds, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  // set once per process (thread-safe initialisation of a local static) to
  // the largest footprint of any op type
  static const hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&k_wave), hipFuncAttributeMaxDynamicSharedMemorySize,
      (int)max_lds_bytes());
  if (attr != hipSuccess) return attr;
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
// `workers` workgroups.  kind 0 runs factor schedules (LDS of the largest
// factor op), kind 1 solve schedules.
static size_t df_lds(int kind) {
  if (kind == 0) return sizeof(hlu::TruncShared);
  size_t m = 0;
  for (int t : {hlu::OP_INVAPPLY, hlu::OP_MVT, hlu::OP_MVROW}) m = std::max(m, hlu::lds_bytes(t));
  return m;
}
static const void* df_kernel(int kind) {
  return kind == 0 ? reinterpret_cast<const void*>(&hlu::k_df_factor)
                   : reinterpret_cast<const void*>(&hlu::k_df_solve);
}
static hipError_t df_attr(int kind) {
  // set once per process and kernel (thread-safe initialisation of local statics)
  static const hipError_t e0 = hipFuncSetAttribute(
      df_kernel(0), hipFuncAttributeMaxDynamicSharedMemorySize, (int)df_lds(0));
  static const hipError_t e1 = hipFuncSetAttribute(
      df_kernel(1), hipFuncAttributeMaxDynamicSharedMemorySize, (int)df_lds(1));
  return kind == 0 ? e0 : e1;
}

// Runs the union of np schedule parts (n ops in all) with `workers`
// persistent workgroups: reset of the in-degrees and the queue (seeded with
// the nready globally numbered ops in ready0), then the executor.  When
// `status` is given, it is cleared first.
extern "C" hipError_t hlu_launch_dataflow(int kind, const void* parts, int np, int* queue,
                                          const int* ready0, int nready, int* ctrl, int n,
                                          int nhigh, int nhw, int workers, long long timeout,
                                          int32_t* status, hipStream_t s) {
  if (kind != 0 && kind != 1) return hipErrorInvalidValue;
  if (nhigh < 0 || nhigh > n - nready || nhw < 0 || (nhigh > 0 && nhw >= workers))
    return hipErrorInvalidValue;
  hipError_t e = df_attr(kind);
  if (e != hipSuccess) return e;
  if (n <= 0) return hipSuccess;
  const hlu::DfPart* pp = reinterpret_cast<const hlu::DfPart*>(parts);
  if (status) hipLaunchKernelGGL(hlu::k_set_int, dim3(1), dim3(64), 0, s, status, 0);
  hipLaunchKernelGGL(hlu::k_df_reset, dim3((n + 255) / 256), dim3(256), 0, s, pp, np, queue, ready0,
                     nready, n, ctrl);
  if (kind == 0)
    hipLaunchKernelGGL(hlu::k_df_factor, dim3(workers), dim3(NT), df_lds(0), s, pp, np, queue,
                       ctrl, n, nhigh, nhw, timeout);
  else
    hipLaunchKernelGGL(hlu::k_df_solve, dim3(workers), dim3(NT), df_lds(1), s, pp, np, queue,
                       ctrl, n, nhigh, nhw, timeout);
  return hipGetLastError();
}

// The same run as a graph (status clear, reset, executor), built explicitly.
extern "C" hipError_t hlu_build_df_graph(int kind, const void* parts, int np, int* queue,
                                         const int* ready0, int nready, int* ctrl, int n,
                                         int nhigh, int nhw, int workers, long long timeout,
                                         int32_t* status, hipGraphExec_t* out) {
  *out = nullptr;
  if (kind != 0 && kind != 1) return hipErrorInvalidValue;
  if (nhigh < 0 || nhigh > n - nready || nhw < 0 || (nhigh > 0 && nhw >= workers))
    return hipErrorInvalidValue;
  hipError_t e = df_attr(kind);
  if (e != hipSuccess) return e;
  hipGraph_t g;
  e = hipGraphCreate(&g, 0);
  if (e != hipSuccess) return e;
  const hlu::DfPart* pp = reinterpret_cast<const hlu::DfPart*>(parts);
  hipGraphNode_t n0, n1, n2;
  if (status) {   // the status word is cleared only when given
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
    void* args[] = {&pp, &np, &queue, &ready0, &nready, &n, &ctrl};
    hipKernelNodeParams p = {};
    p.func = reinterpret_cast<void*>(&hlu::k_df_reset);
    p.gridDim = dim3((n + 255) / 256);
    p.blockDim = dim3(256);
    p.kernelParams = args;
    e = hipGraphAddKernelNode(&n1, g, status ? &n0 : nullptr, status ? 1 : 0, &p);
  }
  if (e == hipSuccess) {
    void* args[] = {&pp, &np, &queue, &ctrl, &n, &nhigh, &nhw, &timeout};
    hipKernelNodeParams p = {};
    p.func = const_cast<void*>(df_kernel(kind));
    p.gridDim = dim3(workers);
    p.blockDim = dim3(NT);
    p.sharedMemBytes = (unsigned)df_lds(kind);
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
                                     (int)hlu::max_lds_bytes());
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

// ---------------------------------------------------------------- construction
// Building the H-matrix on the device from the points (cluster order, x y z
// interleaved, then the panel weights): the dense near field entry by entry,
// each admissible block by adaptive cross approximation with partial
// pivoting (one workgroup per block), recompressed afterwards by the
// truncation kernel.  Entries as in include/hlu.h (kernels of Sec. 6.1).
namespace hlu {

__device__ __forceinline__ double kentry(const double* __restrict__ pts, int npts, int kernel,
                                         int i, int j) {
  const double* a = pts + 3 * (size_t)npts;
  if (i == j) {
    if (kernel == 2) return a[i] * (1.0 - log(0.5 * a[i])) + 1.0;
    if (kernel == 3) return a[i] * (1.0 - log(0.5 * a[i])) * (0.5 / M_PI) + 1.0;
    return 2.0 * sqrt(a[i] / M_PI) / (4.0 * M_PI) * sqrt(M_PI) + 1.0;
  }
  const double dx = pts[3 * i] - pts[3 * j], dy = pts[3 * i + 1] - pts[3 * j + 1],
               dz = pts[3 * i + 2] - pts[3 * j + 2];
  const double r2 = dx * dx + dy * dy + dz * dz;
  if (kernel == 2) return -a[j] * 0.5 * log(r2);
  if (kernel == 3) return -a[j] * 0.5 * log(r2) * (0.5 / M_PI);
  const double g = rsqrt(r2) * (0.25 / M_PI);
  return kernel == 0 ? g * a[j] : g;
}

__global__ void __launch_bounds__(NT) k_asm_dense(const AsmBlock* __restrict__ tab,
                                                  const double* __restrict__ pts, int npts,
                                                  int kernel) {
  const AsmBlock b = tab[blockIdx.x];
  HLU_G double* F = gptr<double>(b.U);
  const int tot = b.m * b.n;
  for (int e = threadIdx.x; e < tot; e += NT) {
    const int i = e % b.m, j = e / b.m;
    F[e] = kentry(pts, npts, kernel, b.r0 + i, b.c0 + j);
  }
}

// block-wide argmax of (v, index) with the smallest index among equal
// values; the result is returned to every thread
__device__ __forceinline__ void block_argmax(double& v, int& ix, double* rv, int* ri) {
  wave_argmax(v, ix);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    rv[w] = v;
    ri[w] = ix;
  }
  __syncthreads();
  v = rv[0];
  ix = ri[0];
  for (int q = 1; q < NT / 64; ++q)
    if (rv[q] > v || (rv[q] == v && ri[q] < ix)) {
      v = rv[q];
      ix = ri[q];
    }
  __syncthreads();
}
__device__ __forceinline__ double block_sum_d(double v, double* rv) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) rv[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < NT / 64; ++q) t += rv[q];
  __syncthreads();
  return t;
}

#define ASM_KMAX 64
#define ASM_MAXDIM 65536
#define LDS_ASM (2 * (ASM_MAXDIM / 32) * 4 + 2 * ASM_KMAX * 8 + 16 * 8 + 16 * 4)
// Adaptive cross approximation with partial pivoting (one block per
// workgroup): step k takes the residual row i of the block, its largest
// entry |.| over the unused columns as pivot (column js), the residual
// column js, and the rank-one term col * row / pivot; the next pivot row is
// the largest entry of that column over the unused rows.  Stops after two
// consecutive terms with |u||v| <= eps |S_k|_F (S_k the current sum, its
// Frobenius norm updated exactly from the new term's inner products), at
// kmax terms (counted in *caphits), or when no usable row is left.  U keeps
// the columns negated on exit.
__global__ void __launch_bounds__(NT) k_asm_aca(const AsmBlock* __restrict__ tab,
                                                const double* __restrict__ pts, int npts,
                                                int kernel, double eps, int kmax,
                                                int32_t* caphits) {
  extern __shared__ __align__(16) char lds[];
  uint32_t* urow = reinterpret_cast<uint32_t*>(lds);
  uint32_t* ucol = urow + ASM_MAXDIM / 32;
  double* bu = reinterpret_cast<double*>(ucol + ASM_MAXDIM / 32);
  double* bv = bu + ASM_KMAX;
  double* rv = bv + ASM_KMAX;
  int* ri = reinterpret_cast<int*>(rv + 16);
  const AsmBlock b = tab[blockIdx.x];
  const int m = b.m, n = b.n, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  HLU_G double* U = gptr<double>(b.U);
  HLU_G double* V = gptr<double>(b.V);
  for (int q = tid; q < (m + 31) / 32; q += NT) urow[q] = 0u;
  for (int q = tid; q < (n + 31) / 32; q += NT) ucol[q] = 0u;
  __syncthreads();
  int k = 0, i = 0, small = 0, zero_tries = 0;
  double norm2 = 0.0;
  kmax = min(kmax, min(min(m, n), ASM_KMAX));
  while (k < kmax) {
    // residual row i -> V[:, k]
    if (tid < k) bu[tid] = U[i + (size_t)tid * m];
    __syncthreads();
    double best = -1.0;
    int js = n;
    for (int j = tid; j < n; j += NT) {
      double v = kentry(pts, npts, kernel, b.r0 + i, b.c0 + j);
      for (int l = 0; l < k; ++l) v -= bu[l] * V[j + (size_t)l * n];
      V[j + (size_t)k * n] = v;
      const bool used = (ucol[j >> 5] >> (j & 31)) & 1u;
      if (!used && fabs(v) > best) {
        best = fabs(v);
        js = j;
      }
    }
    __syncthreads();
    if (tid == 0) urow[i >> 5] |= 1u << (i & 31);
    block_argmax(best, js, rv, ri);
    if (js >= n || !(best > 0.0)) {
      // zero residual row: try the first unused row instead
      int nx = m;
      for (int q = tid; q < m; q += NT)
        if (!((urow[q >> 5] >> (q & 31)) & 1u)) {
          nx = q;
          break;
        }
      double d = -(double)nx;
      block_argmax(d, nx, rv, ri);   // the smallest candidate (largest -q)
      if (nx >= m || ++zero_tries > 3) break;
      i = nx;
      continue;
    }
    if (tid == 0) ucol[js >> 5] |= 1u << (js & 31);
    const double piv = V[js + (size_t)k * n];
    // residual column js -> U[:, k]
    if (tid < k) bv[tid] = V[js + (size_t)tid * n];
    __syncthreads();
    double nu = 0.0, bestc = -1.0;
    int inext = m;
    for (int q = tid; q < m; q += NT) {
      double v = kentry(pts, npts, kernel, b.r0 + q, b.c0 + js);
      for (int l = 0; l < k; ++l) v -= bv[l] * U[q + (size_t)l * m];
      U[q + (size_t)k * m] = v;
      nu += v * v;
      const bool used = (urow[q >> 5] >> (q & 31)) & 1u;
      if (!used && fabs(v) > bestc) {
        bestc = fabs(v);
        inext = q;
      }
    }
    double nv = 0.0;
    const double ip = 1.0 / piv;
    for (int j = tid; j < n; j += NT) {
      const double v = V[j + (size_t)k * n] * ip;
      V[j + (size_t)k * n] = v;
      nv += v * v;
    }
    __syncthreads();   // U[:, k] and V[:, k] complete before other lanes read them
    // cross terms sum_l (u_l . u_k)(v_l . v_k): wavefront w takes l = w, w + 4, ...
    double cross = 0.0;
    for (int l = wid; l < k; l += NT / 64) {
      double a = 0.0, c = 0.0;
      for (int q = lane; q < m; q += 64) a += U[q + (size_t)l * m] * U[q + (size_t)k * m];
      for (int j = lane; j < n; j += 64) c += V[j + (size_t)l * n] * V[j + (size_t)k * n];
      a = wave_sum(a);
      c = wave_sum(c);
      if (lane == 0) cross += a * c;
    }
    nu = block_sum_d(nu, rv);
    nv = block_sum_d(nv, rv);
    cross = block_sum_d(cross, rv);
    norm2 += nu * nv + 2.0 * cross;
    ++k;
    block_argmax(bestc, inext, rv, ri);
    if (sqrt(nu * nv) <= eps * sqrt(fabs(norm2))) {
      if (++small >= 2) break;
    } else {
      small = 0;
    }
    if (inext >= m || !(bestc >= 0.0)) break;
    if (k == kmax && tid == 0) atomicAdd(caphits, 1);
    i = inext;
  }
  for (int e = tid; e < m * k; e += NT) U[e] = -U[e];
  if (tid == 0) *gptr<int32_t>(b.rank) = k;
}

// Y = beta B + alpha A X by direct summation over the exact entries (no
// compression): thread t of workgroup g owns row g * NT + t; the columns go
// by tiles of DMV_TJ points staged in LDS with their X rows.  With absmode,
// Y_i = sum_j |A_ij| (X, B unused).  NRB >= nrhs.
#define DMV_TJ 64
template <int KER, int NRB>
__global__ void __launch_bounds__(NT) k_direct_mv(const double* __restrict__ pts, int npts,
                                                  const double* __restrict__ X, int ldx,
                                                  const double* __restrict__ B, double beta,
                                                  double alpha, double* __restrict__ Y, int nrhs,
                                                  int absmode) {
  __shared__ double sp[DMV_TJ * 4];
  __shared__ double sx[DMV_TJ * (NRB + 1)];
  const int i = blockIdx.x * NT + threadIdx.x;
  const int ii = min(i, npts - 1);
  const double* a = pts + 3 * (size_t)npts;
  const double xi = pts[3 * ii], yi = pts[3 * ii + 1], zi = pts[3 * ii + 2];
  double acc[NRB];
#pragma unroll
  for (int r = 0; r < NRB; ++r) acc[r] = 0.0;
  for (int j0 = 0; j0 < npts; j0 += DMV_TJ) {
    const int nj = min(DMV_TJ, npts - j0);
    for (int e = threadIdx.x; e < DMV_TJ * 4; e += NT) {
      const int jj = e >> 2, c = e & 3, j = j0 + min(jj, nj - 1);
      sp[e] = c < 3 ? pts[3 * j + c] : a[j];
    }
    // X rows of the tile: consecutive threads read consecutive rows of one
    // column (coalesced); padded rows keep the LDS stores conflict-free
    if (!absmode)
      for (int e = threadIdx.x; e < DMV_TJ * NRB; e += NT) {
        const int jj = e % DMV_TJ, r = e / DMV_TJ;
        sx[jj * (NRB + 1) + r] = (jj < nj && r < nrhs) ? X[(j0 + jj) + (size_t)r * ldx] : 0.0;
      }
    __syncthreads();
    for (int jj = 0; jj < nj; ++jj) {
      const int j = j0 + jj;
      double g;
      if (j == ii) {
        g = kentry(pts, npts, KER, ii, ii);
      } else {
        const double dx = xi - sp[4 * jj], dy = yi - sp[4 * jj + 1], dz = zi - sp[4 * jj + 2];
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (KER == 2) g = -sp[4 * jj + 3] * 0.5 * log(r2);
        else if (KER == 3) g = -sp[4 * jj + 3] * 0.5 * log(r2) * (0.5 / M_PI);
        else if (KER == 0) g = rsqrt(r2) * (0.25 / M_PI) * sp[4 * jj + 3];
        else g = rsqrt(r2) * (0.25 / M_PI);
      }
      if (absmode) {
        acc[0] += fabs(g);
      } else {
#pragma unroll
        for (int r = 0; r < NRB; ++r) acc[r] += g * sx[jj * (NRB + 1) + r];
      }
    }
    __syncthreads();
  }
  if (i < npts) {
    if (absmode) {
      Y[i] = acc[0];
    } else {
      // unrolled with a guard (a loop to nrhs would index acc dynamically
      // and move it to scratch memory)
#pragma unroll
      for (int r = 0; r < NRB; ++r)
        if (r < nrhs) {
          const double bv = beta != 0.0 ? beta * B[i + (size_t)r * ldx] : 0.0;
          Y[i + (size_t)r * ldx] = bv + alpha * acc[r];
        }
    }
  }
}

}  // namespace hlu

extern "C" size_t hlu_asm_lds_bytes(void) { return LDS_ASM; }

extern "C" hipError_t hlu_launch_asm(const void* dense, int ndense, const void* lr, int nlr,
                                     const double* pts, int npts, int kernel, double eps,
                                     int kmax, int32_t* caphits, hipStream_t s) {
  static const hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&hlu::k_asm_aca), hipFuncAttributeMaxDynamicSharedMemorySize,
      (int)LDS_ASM);
  if (attr != hipSuccess) return attr;
  if (ndense > 0)
    hipLaunchKernelGGL(hlu::k_asm_dense, dim3(ndense), dim3(NT), 0, s,
                       reinterpret_cast<const hlu::AsmBlock*>(dense), pts, npts, kernel);
  if (nlr > 0)
    hipLaunchKernelGGL(hlu::k_asm_aca, dim3(nlr), dim3(NT), LDS_ASM, s,
                       reinterpret_cast<const hlu::AsmBlock*>(lr), pts, npts, kernel, eps, kmax,
                       caphits);
  return hipGetLastError();
}

template <int KER>
static void launch_dmv(dim3 g, const double* pts, int npts, const double* X, int ldx,
                       const double* B, double beta, double alpha, double* Y, int nrhs,
                       int absmode, hipStream_t s) {
  if (absmode || nrhs <= 4)
    hipLaunchKernelGGL((hlu::k_direct_mv<KER, 4>), g, dim3(NT), 0, s, pts, npts, X, ldx, B, beta,
                       alpha, Y, nrhs, absmode);
  else if (nrhs <= 16)
    hipLaunchKernelGGL((hlu::k_direct_mv<KER, 16>), g, dim3(NT), 0, s, pts, npts, X, ldx, B,
                       beta, alpha, Y, nrhs, absmode);
  else if (nrhs <= 32)
    hipLaunchKernelGGL((hlu::k_direct_mv<KER, 32>), g, dim3(NT), 0, s, pts, npts, X, ldx, B,
                       beta, alpha, Y, nrhs, absmode);
  else
    hipLaunchKernelGGL((hlu::k_direct_mv<KER, 64>), g, dim3(NT), 0, s, pts, npts, X, ldx, B,
                       beta, alpha, Y, nrhs, absmode);
}

// Y = beta B + alpha A X (n x nrhs, leading dimension ld, nrhs <= 64) with
// the exact matrix by direct summation; absmode: Y = |A| 1 (nrhs ignored).
extern "C" hipError_t hlu_launch_direct_mv(const double* pts, int npts, int kernel,
                                           const double* X, int ld, const double* B, double beta,
                                           double alpha, double* Y, int nrhs, int absmode,
                                           hipStream_t s) {
  if (npts <= 0) return hipSuccess;
  if (nrhs > 64 || kernel < 0 || kernel > 3) return hipErrorInvalidValue;
  dim3 g((npts + NT - 1) / NT);
  switch (kernel) {
    case 0: launch_dmv<0>(g, pts, npts, X, ld, B, beta, alpha, Y, nrhs, absmode, s); break;
    case 1: launch_dmv<1>(g, pts, npts, X, ld, B, beta, alpha, Y, nrhs, absmode, s); break;
    case 2: launch_dmv<2>(g, pts, npts, X, ld, B, beta, alpha, Y, nrhs, absmode, s); break;
    default: launch_dmv<3>(g, pts, npts, X, ld, B, beta, alpha, Y, nrhs, absmode, s); break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- static scratch
// Staging of the allocation-free truncation entry point: one truncation
// descriptor and its term table, written by a small kernel from scalar
// arguments, live in this file-scope array instead of an allocation.  Every
// device keeps its own copy for the life of the process.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for
// the symbol): it uses the address hipGetSymbolAddress returns on the device
// in question, looked up once per device on the entry point's first call
// there.
#define HLU_STATIC_SCRATCH_BYTES 4096
static __device__ __align__(256) char scratch[HLU_STATIC_SCRATCH_BYTES];

namespace hlu {
// Op at dst, term t at dst + sizeof(Op) + t * sizeof(Term): term t covers
// the columns [t w, min(kx, (t + 1) w)) of X (m x kx) and Y (n x kx).
__global__ void k_build_trunc(char* dst, uint64_t U, uint64_t V, uint64_t rank, uint64_t X,
                              uint64_t Y, int m, int n, int kx, int w, int cap, double eps,
                              int fixed_rank) {
  const int t = threadIdx.x;
  const int nt = (kx + w - 1) / w;
  Term* terms = reinterpret_cast<Term*>(dst + sizeof(Op));
  if (t < nt) {
    Term tm;
    const int c0 = t * w, cw = min(w, kx - c0);
    tm.X = PRef{X + (uint64_t)c0 * m * 8, 0, m, m, cw, DT_F64, 0, PK_MAT, 0};
    tm.Y = PRef{Y + (uint64_t)c0 * n * 8, 0, n, n, cw, DT_F64, 0, PK_MAT, 0};
    tm.xo = 0;
    tm.yo = 0;
    tm.pad[0] = tm.pad[1] = 0;
    terms[t] = tm;
  }
  if (t == 0) {
    Op o;
    o.type = OP_TRUNC;
    o.i0 = 0;
    o.i1 = nt;
    o.i2 = cap | (fixed_rank << 16);
    o.d0 = eps;
    o.cost = 0;
    o.p[0] = PRef{U, rank, m, m, cap, DT_F64, 0, PK_MAT, 0};
    o.p[1] = PRef{V, rank, n, n, cap, DT_F64, 0, PK_MAT, 0};
    o.p[2] = PRef{(uint64_t)terms, 0, 0, 0, 0, DT_F64, 0, PK_MAT, 0};
    o.p[3] = PRef{0, 0, 0, 0, 0, DT_F64, 0, PK_MAT, 0};
    *reinterpret_cast<Op*>(dst) = o;
  }
}
}  // namespace hlu

extern "C" size_t hlu_static_scratch_bytes(void) { return HLU_STATIC_SCRATCH_BYTES; }

// Device address of `scratch` on the current device (looked up once per
// device; later calls return the kept address).
extern "C" hipError_t hlu_static_scratch(void** out) {
  static std::mutex mu;
  static std::map<int, void*> addr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    it = addr.emplace(dev, ptr).first;
  }
  *out = it->second;
  return hipSuccess;
}

extern "C" hipError_t hlu_launch_build_trunc(void* dst, const double* U, const double* V,
                                             int32_t* rank, const double* X, const double* Y, int m,
                                             int n, int kx, int w, int cap, double eps,
                                             int fixed_rank, hipStream_t s) {
  hipLaunchKernelGGL(hlu::k_build_trunc, dim3(1), dim3(64), 0, s, (char*)dst, (uint64_t)U,
                     (uint64_t)V, (uint64_t)rank, (uint64_t)X, (uint64_t)Y, m, n, kx, w, cap, eps,
                     fixed_rank);
  return hipGetLastError();
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

extern "C" hipError_t hlu_launch_axpy_masked(const double* d, double* x, int ld, int n, int nrhs,
                                             const int32_t* active, hipStream_t s) {
  int64_t tot = (int64_t)n * nrhs;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(hlu::k_axpy_masked, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, x, d,
                     ld, n, nrhs, active);
  return hipGetLastError();
}

extern "C" hipError_t hlu_launch_colmax(const double* R, const double* X, const double* B, int ld,
                                        int n, int nrhs, double* out, hipStream_t s) {
  hipLaunchKernelGGL(hlu::k_colmax, dim3(nrhs), dim3(NT), 0, s, R, X, B, ld, n, out);
  return hipGetLastError();
}

extern "C" hipError_t hlu_launch_keep_flag(const int32_t* src, int32_t* dst, hipStream_t s) {
  hipLaunchKernelGGL(hlu::k_keep_flag, dim3(1), dim3(64), 0, s, src, dst);
  return hipGetLastError();
}

extern "C" hipError_t hlu_launch_set_int(int32_t* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(hlu::k_set_int, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}
