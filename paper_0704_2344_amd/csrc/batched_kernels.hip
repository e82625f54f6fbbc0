// Batched right-hand sides: the block-sparse matrix times a dense block of up
// to 64 columns (SpMM), and per-column COCG steps.  Each column keeps its
// iterate and residual recurrence in FP64; only the directions P are stored
// in complex64.  The product Q = A P is formed in FP64 arithmetic and kept
// in FP64: summing a row's 81 complex terms in FP32 perturbs the product by
// enough to destroy the conjugacy of the directions on large indefinite
// systems (the columns then stagnate), while rounding only the directions
// to complex64 costs a few percent of iterations.
//
// Layout: a block vector is [n_unknowns][64] (column fastest), so the 64
// columns of one unknown are contiguous and a wavefront with lane = column
// reads them in one coalesced access.
//
// Two SpMM kernels, chosen by timing:
//  * vector FMAs: the complex128 matrix times the promoted complex64
//    directions, FP64 FMAs, lane = column;
//  * matrix cores: v_mfma_f32_4x4x1_16b_f32 computes 16 independent 4x4x1
//    outer products: lane l supplies A of block l/4 row l%4 and B of block
//    l/4 column l%4, and receives C of block l/4 column l%4 in its four
//    accumulator registers (rows 0..3).  With the block index = column
//    group, lane l owns RHS column l and the registers hold the three row
//    components (row 3 is padding).  Each complex 3x3 block times the
//    column's three components takes four MFMAs per component (Ar Xr, Ai Xi,
//    Ar Xi, Ai Xr) on the complex64 matrix in FP32; the block's result is
//    then added into FP64 row accumulators, so FP32 rounding never sees
//    more than one block's three terms.
//
// Per-column dot products are written as per-workgroup partials and summed
// in a fixed order by a separate per-column reduction kernel.
#include "internal.h"

namespace femh {
namespace {

constexpr int kLD = 64;           // column stride of block vectors
constexpr int kBT = 256;          // threads per workgroup (4 waves)

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Rows are dealt to waves so each XCD (round-robin workgroup dispatch over 8)
// sweeps a contiguous window of rows.
__device__ __forceinline__ int wave_index(int waves_per_block, int& nwaves) {
  const int wib = threadIdx.x >> 6;
  const int xcd = blockIdx.x & 7;
  const int loc = blockIdx.x >> 3;
  const int per_xcd = gridDim.x >> 3;
  nwaves = gridDim.x * waves_per_block;
  return (xcd * per_xcd + loc) * waves_per_block + wib;
}

// Per-column partial sums of p^T q (re, im), ||p||^2, ||q||^2 over the
// workgroup -> partials[block][col][4].
__device__ __forceinline__ void store_col_partials(const double (&v)[4], double* __restrict__ partials) {
  __shared__ double s[kBT / 64][64][4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k) s[wid][lane][k] = v[k];
  __syncthreads();
  if (threadIdx.x < 64 * 4) {
    const int col = threadIdx.x >> 2, k = threadIdx.x & 3;
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kBT / 64; ++w) t += s[w][col][k];
    partials[((size_t)blockIdx.x * 64 + col) * 4 + k] = t;
  }
}

// Per-column p^T q, ||p||^2, ||q||^2 of one row component.
__device__ __forceinline__ void pq_terms(const float2 p, double yr, double yi, double (&acc)[4]) {
  acc[0] += (double)p.x * yr - (double)p.y * yi;
  acc[1] += (double)p.x * yi + (double)p.y * yr;
  acc[2] += (double)p.x * p.x + (double)p.y * p.y;
  acc[3] += yr * yr + yi * yi;
}

// Q = A P on the matrix cores (complex64 matrix, FP32 products per block,
// FP64 sum over blocks), with per-column p^T q.
__global__ void __launch_bounds__(kBT) k_bspmm_mfma(PatternDev pt, const float2* __restrict__ val,
                                                    const float2* __restrict__ P, double2* __restrict__ Q,
                                                    double* __restrict__ partials, const BatchScalars* sc) {
  if (sc->active == 0) return;
  const int lane = threadIdx.x & 63;
  const int m = lane & 3;  // A row supplied by this lane
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int nwaves;
  for (int r = wave_index(kBT / 64, nwaves); r < pt.nn; r += nwaves) {
    const int beg = uniform_int(pt.row_ptr[r]);
    const int end = uniform_int(pt.row_ptr[r + 1]);
    double yr[3] = {0.0, 0.0, 0.0}, yi[3] = {0.0, 0.0, 0.0};
    for (int b = beg; b < end; ++b) {
      const int c = uniform_int(pt.col_idx[b]);
      const float2* blk = val + (size_t)b * 9;
      const float2* xrow = P + (size_t)3 * c * kLD + lane;
      v4f K1 = {0.f, 0.f, 0.f, 0.f}, K2 = K1, K3 = K1, K4 = K1;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const float2 a = m < 3 ? blk[3 * m + j] : make_float2(0.f, 0.f);
        const float2 x = xrow[j * kLD];
        K1 = __builtin_amdgcn_mfma_f32_4x4x1f32(a.x, x.x, K1, 0, 0, 0);
        K2 = __builtin_amdgcn_mfma_f32_4x4x1f32(a.y, x.y, K2, 0, 0, 0);
        K3 = __builtin_amdgcn_mfma_f32_4x4x1f32(a.x, x.y, K3, 0, 0, 0);
        K4 = __builtin_amdgcn_mfma_f32_4x4x1f32(a.y, x.x, K4, 0, 0, 0);
      }
      // lane = column; register i = row component
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        yr[i] += (double)K1[i] - (double)K2[i];
        yi[i] += (double)K3[i] + (double)K4[i];
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const size_t idx = (size_t)(3 * r + i) * kLD + lane;
      Q[idx] = make_double2(yr[i], yi[i]);
      pq_terms(P[idx], yr[i], yi[i], acc);
    }
  }
  store_col_partials(acc, partials);
}

// Same product with FP64 vector FMAs on the complex128 matrix (lane = column).
// The row's column indices (at most 27) come in with one vector load and are
// taken lane by lane with readlane, so each block costs one memory latency
// (its x entries and its matrix values load together) instead of two.
__global__ void __launch_bounds__(kBT) k_bspmm_vec(PatternDev pt, const double2* __restrict__ val,
                                                   const float2* __restrict__ P, double2* __restrict__ Q,
                                                   double* __restrict__ partials, const BatchScalars* sc) {
  if (sc->active == 0) return;
  const int lane = threadIdx.x & 63;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int nwaves;
  for (int r = wave_index(kBT / 64, nwaves); r < pt.nn; r += nwaves) {
    const int beg = uniform_int(pt.row_ptr[r]);
    const int end = uniform_int(pt.row_ptr[r + 1]);
    const int cl = lane < end - beg ? pt.col_idx[beg + lane] : 0;
    double yr[3] = {0.0, 0.0, 0.0}, yi[3] = {0.0, 0.0, 0.0};
    for (int b = beg; b < end; ++b) {
      const int c = __builtin_amdgcn_readlane(cl, b - beg);
      const double2* blk = val + (size_t)b * 9;
      const float2* xrow = P + (size_t)3 * c * kLD + lane;
      const float2 f0 = xrow[0], f1 = xrow[kLD], f2 = xrow[2 * kLD];
      const double2 x0 = make_double2(f0.x, f0.y), x1 = make_double2(f1.x, f1.y), x2 = make_double2(f2.x, f2.y);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double2 a0 = blk[3 * i], a1 = blk[3 * i + 1], a2 = blk[3 * i + 2];
        yr[i] += a0.x * x0.x - a0.y * x0.y + a1.x * x1.x - a1.y * x1.y + a2.x * x2.x - a2.y * x2.y;
        yi[i] += a0.x * x0.y + a0.y * x0.x + a1.x * x1.y + a1.y * x1.x + a2.x * x2.y + a2.y * x2.x;
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const size_t idx = (size_t)(3 * r + i) * kLD + lane;
      Q[idx] = make_double2(yr[i], yi[i]);
      pq_terms(P[idx], yr[i], yi[i], acc);
    }
  }
  store_col_partials(acc, partials);
}

// ------------------------------------------------ per-column reductions
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double s = fmax(fabs(b.x), fabs(b.y));
  const double br = b.x / s, bi = b.y / s;
  const double d = br * br + bi * bi;
  return make_double2((a.x * br + a.y * bi) / (d * s), (a.y * br - a.x * bi) / (d * s));
}
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// Sum partials[b][col][0..3] over b in fixed order: one workgroup per column.
__device__ __forceinline__ void column_total(const double* __restrict__ partials, int nblocks, int col,
                                             double (&tot)[4]) {
  __shared__ double s[kBT][4];
  double v[4] = {0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += kBT)
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] += partials[((size_t)b * 64 + col) * 4 + k];
#pragma unroll
  for (int k = 0; k < 4; ++k) s[threadIdx.x][k] = v[k];
  __syncthreads();
  for (int w = kBT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < 4; ++k) s[threadIdx.x][k] += s[threadIdx.x + w][k];
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) tot[k] = s[0][k];
}

// After the product: alpha_c = rho_c / p_c^T q_c.
__global__ void __launch_bounds__(kBT) k_bred_alpha(const double* __restrict__ partials, int nblocks, BatchScalars* sc) {
  if (sc->active == 0) return;
  const int col = blockIdx.x;
  double t[4];
  column_total(partials, nblocks, col, t);
  if (threadIdx.x == 0 && sc->done[col] == 0) {
    const double2 pq = make_double2(t[0], t[1]);
    if (cabs2(pq) <= sc->bd_tol * sc->bd_tol * t[2] * t[3]) {
      sc->done[col] = 3;
      sc->alpha[col] = make_double2(0.0, 0.0);
    } else {
      sc->alpha[col] = cdiv(sc->rho[col], pq);
    }
  }
}

// After the update: convergence, iteration limit, breakdown, reliable-update
// trigger, beta_c.  The last workgroup recounts the active columns.
__global__ void __launch_bounds__(kBT) k_bred_beta(const double* __restrict__ partials, int nblocks, BatchScalars* sc) {
  if (sc->active == 0) return;
  const int col = blockIdx.x;
  double t[4];
  column_total(partials, nblocks, col, t);
  __shared__ int s_last;
  if (threadIdx.x == 0) {
    if (sc->done[col] == 0) {
      const double2 rho_new = make_double2(t[0], t[1]);
      const double rr = t[2], zz = t[3];
      sc->iters[col] += 1;
      sc->rr[col] = rr;
      if (rr <= sc->tol2[col]) {
        sc->done[col] = 1;
      } else if (sc->iters[col] >= sc->max_iters) {
        sc->done[col] = 2;
      } else if (cabs2(rho_new) <= sc->bd_tol * sc->bd_tol * rr * zz) {
        sc->done[col] = 3;
      } else {
        bool trigger = false;
        if (rr > sc->rr_max[col]) sc->rr_max[col] = rr;
        else trigger = rr <= sc->delta2 * sc->rr_max[col];
        if (trigger) {
          sc->done[col] = 4;
        } else {
          sc->beta[col] = cdiv(rho_new, sc->rho[col]);
          sc->rho[col] = rho_new;
        }
      }
    }
    __threadfence();
    s_last = atomicAdd(&sc->ticket, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (s_last && threadIdx.x == 0) {
    __threadfence();
    int act = 0;
    for (int c = 0; c < (int)gridDim.x; ++c)
      act += __hip_atomic_load(&sc->done[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    sc->active = act;
    sc->ticket = 0u;
  }
}

// x += alpha p; r -= alpha q (FP64); z = D^-1 r; per-column rho', ||r||^2,
// ||z||^2.
__global__ void __launch_bounds__(kBT) k_bupdate(int64_t n, const double2* __restrict__ dinv, double2* __restrict__ X,
                                                 double2* __restrict__ R, const float2* __restrict__ P,
                                                 const double2* __restrict__ Q, double* __restrict__ partials,
                                                 const BatchScalars* sc) {
  if (sc->active == 0) return;
  const int col = threadIdx.x & 63;
  const bool on = sc->done[col] == 0;
  const double ar = sc->alpha[col].x, ai = sc->alpha[col].y;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t rows_per_block = kBT / 64;
  for (int64_t u = (int64_t)blockIdx.x * rows_per_block + (threadIdx.x >> 6); u < n;
       u += (int64_t)gridDim.x * rows_per_block) {
    if (!on) continue;
    const size_t idx = (size_t)u * kLD + col;
    const float2 p = P[idx];
    const double2 q = Q[idx];
    const double2 d = dinv[u];
    double2 x = X[idx];
    double2 r = R[idx];
    x.x += ar * (double)p.x - ai * (double)p.y;
    x.y += ar * (double)p.y + ai * (double)p.x;
    r.x -= ar * q.x - ai * q.y;
    r.y -= ar * q.y + ai * q.x;
    X[idx] = x;
    R[idx] = r;
    const double zr = d.x * r.x - d.y * r.y, zi = d.x * r.y + d.y * r.x;
    v[0] += r.x * zr - r.y * zi;
    v[1] += r.x * zi + r.y * zr;
    v[2] += r.x * r.x + r.y * r.y;
    v[3] += zr * zr + zi * zi;
  }
  store_col_partials(v, partials);
}

// p = D^-1 r + beta p (direction kept in complex64) for running columns,
// or for the columns with only[c] == 1 right after a reliable update.
__global__ void __launch_bounds__(kBT) k_bpupdate(int64_t n, const double2* __restrict__ dinv,
                                                  const double2* __restrict__ R, float2* __restrict__ P,
                                                  const BatchScalars* sc, const int32_t* __restrict__ only) {
  if (sc->active == 0 && !only) return;
  const int col = threadIdx.x & 63;
  const bool on = only ? only[col] == 1 : sc->done[col] == 0;
  if (!on) return;
  const double br = sc->beta[col].x, bi = sc->beta[col].y;
  const int64_t rows_per_block = kBT / 64;
  for (int64_t u = (int64_t)blockIdx.x * rows_per_block + (threadIdx.x >> 6); u < n;
       u += (int64_t)gridDim.x * rows_per_block) {
    const size_t idx = (size_t)u * kLD + col;
    const double2 d = dinv[u], r = R[idx];
    const float2 p = P[idx];
    const double zr = d.x * r.x - d.y * r.y, zi = d.x * r.y + d.y * r.x;
    const double nr = zr + br * p.x - bi * p.y;
    const double ni = zi + br * p.y + bi * p.x;
    P[idx] = make_float2((float)nr, (float)ni);
  }
}

// ------------------------------------------------------------ FP64 parts
// R = B - A X in FP64 (vector FMAs, lane = column) with per-column ||R||^2.
// R = B - A X in FP64 for the columns with mask[c] != 0 (all when mask is
// null); per-column ||B - A X||^2 for every column.
__global__ void __launch_bounds__(kBT) k_bresidual64(PatternDev pt, const double2* __restrict__ val,
                                                     const double2* __restrict__ X, const double2* __restrict__ B,
                                                     double2* __restrict__ R, double* __restrict__ partials,
                                                     const int32_t* __restrict__ mask) {
  const int lane = threadIdx.x & 63;
  const bool store = mask ? mask[lane] != 0 : true;
  double acc = 0.0;
  int nwaves;
  for (int r = wave_index(kBT / 64, nwaves); r < pt.nn; r += nwaves) {
    const int beg = uniform_int(pt.row_ptr[r]);
    const int end = uniform_int(pt.row_ptr[r + 1]);
    double yr[3] = {0, 0, 0}, yi[3] = {0, 0, 0};
    for (int b = beg; b < end; ++b) {
      const int c = uniform_int(pt.col_idx[b]);
      const double2* blk = val + (size_t)b * 9;
      const double2* xrow = X + (size_t)3 * c * kLD + lane;
      const double2 x0 = xrow[0], x1 = xrow[kLD], x2 = xrow[2 * kLD];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double2 a0 = blk[3 * i], a1 = blk[3 * i + 1], a2 = blk[3 * i + 2];
        yr[i] += a0.x * x0.x - a0.y * x0.y + a1.x * x1.x - a1.y * x1.y + a2.x * x2.x - a2.y * x2.y;
        yi[i] += a0.x * x0.y + a0.y * x0.x + a1.x * x1.y + a1.y * x1.x + a2.x * x2.y + a2.y * x2.x;
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const size_t idx = (size_t)(3 * r + i) * kLD + lane;
      const double2 b = B[idx];
      const double2 rv = make_double2(b.x - yr[i], b.y - yi[i]);
      if (store) R[idx] = rv;
      acc += rv.x * rv.x + rv.y * rv.y;
    }
  }
  __shared__ double s[kBT / 64][64];
  s[threadIdx.x >> 6][lane] = acc;
  __syncthreads();
  if (threadIdx.x < 64) {
    double t = 0.0;
    for (int w = 0; w < kBT / 64; ++w) t += s[w][threadIdx.x];
    partials[(size_t)blockIdx.x * 64 + threadIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kBT) k_bred_norm64(const double* __restrict__ partials, int nblocks,
                                                     double* __restrict__ rr64) {
  const int col = blockIdx.x;
  __shared__ double s[kBT];
  double v = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kBT) v += partials[(size_t)b * 64 + col];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int w = kBT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) rr64[col] = s[0];
}

// Reliable update of flagged columns whose residual was just replaced by
// the true one: rho' = r^T D^-1 r; restarting columns (action 2) take
// p = D^-1 r.  Per-column rho', ||r||^2, ||z||^2 partials.
__global__ void __launch_bounds__(kBT) k_brescale(int64_t n, const double2* __restrict__ R,
                                                  const double2* __restrict__ dinv, float2* __restrict__ P,
                                                  double* __restrict__ partials, const BatchPlan* __restrict__ plan) {
  const int col = threadIdx.x & 63;
  const int act = plan->action[col];
  const bool on = act == 1 || act == 2;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t rows_per_block = kBT / 64;
  if (on) {
    for (int64_t u = (int64_t)blockIdx.x * rows_per_block + (threadIdx.x >> 6); u < n;
         u += (int64_t)gridDim.x * rows_per_block) {
      const size_t idx = (size_t)u * kLD + col;
      const double2 r = R[idx];
      const double2 d = dinv[u];
      const double zr = d.x * r.x - d.y * r.y, zi = d.x * r.y + d.y * r.x;
      if (act == 2) P[idx] = make_float2((float)zr, (float)zi);
      v[0] += r.x * zr - r.y * zi;
      v[1] += r.x * zi + r.y * zr;
      v[2] += r.x * r.x + r.y * r.y;
      v[3] += zr * zr + zi * zi;
    }
  }
  store_col_partials(v, partials);
}

__global__ void __launch_bounds__(kBT) k_bred_rescale(const double* __restrict__ partials, int nblocks,
                                                      BatchScalars* sc, const BatchPlan* __restrict__ plan) {
  const int col = blockIdx.x;
  const int act = plan->action[col];
  if (act != 1 && act != 2) {
    if (threadIdx.x == 0 && act == 3) sc->done[col] = plan->final_state[col];
    return;
  }
  double t[4];
  column_total(partials, nblocks, col, t);
  if (threadIdx.x == 0) {
    const double2 rho_new = make_double2(t[0], t[1]);
    const double rr = t[2], zz = t[3];
    sc->tol2[col] = plan->tol2[col];
    sc->rr[col] = rr;
    sc->rr_max[col] = rr;
    sc->done[col] = 0;
    if (cabs2(rho_new) <= sc->bd_tol * sc->bd_tol * rr * zz) {
      sc->done[col] = 3;
    } else if (act == 1) {
      sc->beta[col] = cdiv(rho_new, sc->rho[col]);
    }
    sc->rho[col] = rho_new;
  }
}

__global__ void k_bcount_active(BatchScalars* sc, int ncols) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int act = 0;
    for (int c = 0; c < ncols; ++c) act += sc->done[c] == 0;
    sc->active = act;
  }
}

// [nrhs][n] column-major right-hand sides -> [n][64] block layout (zero pad).
__global__ void k_to_block(int64_t n, int nrhs, const double2* __restrict__ b, double2* __restrict__ B) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * kLD) return;
  const int64_t u = t / kLD;
  const int col = (int)(t % kLD);
  B[t] = col < nrhs ? b[(size_t)col * n + u] : make_double2(0.0, 0.0);
}

// [n][64] block layout -> [nrhs][n]
__global__ void k_from_block(int64_t n, int nrhs, const double2* __restrict__ X, double2* __restrict__ x) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nrhs) return;
  const int64_t r = t / n;
  const int64_t u = t % n;
  x[t] = X[(size_t)u * kLD + r];
}

}  // namespace

namespace k {

int batched_blocks_for(int32_t nn, int n_cu, int per_cu) {
  int64_t b = ((int64_t)nn + 3) / 4;
  int64_t cap = (int64_t)n_cu * per_cu;
  if (cap > 2048) cap = 2048;
  if (b > cap) b = cap;
  if (b < 8) b = 8;
  return (int)((b + 7) / 8 * 8);
}

int batched_vec_blocks(int64_t n) {
  int64_t b = (n + 3) / 4;
  if (b > 2048) b = 2048;
  if (b < 8) b = 8;
  return (int)b;
}

hipError_t bspmm(hipStream_t st, const PatternDev& pt, const double2* val64, const float2* val32, const float2* P,
                 double2* Q, double* partials, const BatchScalars* sc, BatchTile tile) {
  if (tile.kind == 1)
    hipLaunchKernelGGL(k_bspmm_mfma, dim3(tile.blocks), dim3(kBT), 0, st, pt, val32, P, Q, partials, sc);
  else
    hipLaunchKernelGGL(k_bspmm_vec, dim3(tile.blocks), dim3(kBT), 0, st, pt, val64, P, Q, partials, sc);
  return hipGetLastError();
}

hipError_t bred_alpha(hipStream_t st, const double* partials, int nblocks, int ncols, BatchScalars* sc) {
  hipLaunchKernelGGL(k_bred_alpha, dim3(ncols), dim3(kBT), 0, st, partials, nblocks, sc);
  return hipGetLastError();
}

hipError_t bupdate(hipStream_t st, int64_t n, const double2* dinv, double2* X, double2* R, const float2* P,
                   const double2* Q, double* partials, int blocks, const BatchScalars* sc) {
  hipLaunchKernelGGL(k_bupdate, dim3(blocks), dim3(kBT), 0, st, n, dinv, X, R, P, Q, partials, sc);
  return hipGetLastError();
}

hipError_t bred_beta(hipStream_t st, const double* partials, int nblocks, int ncols, BatchScalars* sc) {
  hipLaunchKernelGGL(k_bred_beta, dim3(ncols), dim3(kBT), 0, st, partials, nblocks, sc);
  return hipGetLastError();
}

hipError_t bpupdate(hipStream_t st, int64_t n, const double2* dinv, const double2* R, float2* P, int blocks,
                    const BatchScalars* sc, const int32_t* only) {
  hipLaunchKernelGGL(k_bpupdate, dim3(blocks), dim3(kBT), 0, st, n, dinv, R, P, sc, only);
  return hipGetLastError();
}

hipError_t bresidual64(hipStream_t st, const PatternDev& pt, const double2* val, const double2* X,
                       const double2* B, double2* R, double* partials, int blocks, int ncols, double* rr64,
                       const int32_t* mask) {
  hipLaunchKernelGGL(k_bresidual64, dim3(blocks), dim3(kBT), 0, st, pt, val, X, B, R, partials, mask);
  hipLaunchKernelGGL(k_bred_norm64, dim3(ncols), dim3(kBT), 0, st, (const double*)partials, blocks, rr64);
  return hipGetLastError();
}

hipError_t brescale(hipStream_t st, int64_t n, const double2* R, const double2* dinv, float2* P,
                    double* partials, int blocks, int ncols, BatchScalars* sc, const BatchPlan* plan) {
  hipLaunchKernelGGL(k_brescale, dim3(blocks), dim3(kBT), 0, st, n, R, dinv, P, partials, plan);
  hipLaunchKernelGGL(k_bred_rescale, dim3(ncols), dim3(kBT), 0, st, (const double*)partials, blocks, sc, plan);
  hipLaunchKernelGGL(k_bcount_active, dim3(1), dim3(64), 0, st, sc, ncols);
  return hipGetLastError();
}

hipError_t to_block(hipStream_t st, int64_t n, int nrhs, const double2* b, double2* B) {
  const int64_t t = n * 64;
  hipLaunchKernelGGL(k_to_block, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, n, nrhs, b, B);
  return hipGetLastError();
}

hipError_t from_block(hipStream_t st, int64_t n, int nrhs, const double2* X, double2* x) {
  const int64_t t = n * nrhs;
  hipLaunchKernelGGL(k_from_block, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, n, nrhs, X, x);
  return hipGetLastError();
}

}  // namespace k
}  // namespace femh
