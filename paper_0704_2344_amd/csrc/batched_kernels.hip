// Batched right-hand sides: the block-sparse matrix times a dense block of up
// to 64 columns (SpMM), and per-column COCG steps.  Every column's iterate,
// residual, direction and product are FP64; the matrix in the product is
// the complex128 one or the complex64 one promoted inside FP64 arithmetic.
// Summing a row's 81 complex terms in FP32 perturbs the product by enough
// to destroy the conjugacy of the directions on large indefinite systems
// (columns stagnate), and even storing only the directions in complex64
// makes the recurrence fragile (iteration counts up 40 %, some columns
// several times more).  With 64 columns the vectors carry most of an
// iteration's bytes, so the complex64 matrix saves little there, while its
// perturbation of the operator lengthens some columns' convergence
// several-fold.
//
// Layout: a block vector is [n_unknowns][LD] (column fastest) with LD = 64
// (wide) or LD = 4 (narrow, up to four right-hand sides).  The elementwise
// kernels map lane l to column l % LD of row slot l / LD, so a wavefront
// covers 64 / LD unknowns and reads their columns in coalesced accesses.
//
// Narrow SpMM: the single-RHS SpMV's mapping (one block row per wave, lane
// l < 63 owns entry l % 9 of blocks l / 9 + 7 k) with each loaded matrix
// value applied to all LD columns, so the matrix is read once for the batch.
//
// Two wide SpMM kernels, chosen by timing:
//  * vector FMAs: the promoted complex64 matrix times the FP64 directions,
//    FP64 FMAs, lane = column;
//  * matrix cores: v_mfma_f32_4x4x1_16b_f32 computes 16 independent 4x4x1
//    outer products: lane l supplies A of block l/4 row l%4 and B of block
//    l/4 column l%4, and receives C of block l/4 column l%4 in its four
//    accumulator registers (rows 0..3).  With the block index = column
//    group, lane l owns RHS column l and the registers hold the three row
//    components (row 3 is padding).  Each complex 3x3 block times the
//    column's three components takes four MFMAs per component (Ar Xr, Ai Xi,
//    Ar Xi, Ai Xr) on the complex64 matrix and the directions rounded to
//    FP32; the block's result is then added into FP64 row accumulators, so
//    FP32 rounding never sees more than one block's three terms.
//
// Per-column dot products are written as per-workgroup partials and summed
// in a fixed order by a separate per-column reduction kernel.
#include "internal.h"

namespace femh {
namespace {

constexpr int kLD = 64;           // column stride of the wide layout
constexpr int kBT = 256;          // threads per workgroup (4 waves)

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Matrix value in FP64 arithmetic: complex64 values are promoted exactly.
__device__ __forceinline__ double2 as_f64(float2 f) { return make_double2(f.x, f.y); }
__device__ __forceinline__ double2 as_f64(double2 d) { return d; }

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

// Per-column partial sums of four values over the workgroup ->
// partials[block][col][4]; lane l holds column l % LD.  Fixed summation
// order (threads col, col + LD, ...).
template <int LD>
__device__ __forceinline__ void store_col_partials(const double (&v)[4], double* __restrict__ partials) {
  __shared__ double s[kBT][4];
#pragma unroll
  for (int k = 0; k < 4; ++k) s[threadIdx.x][k] = v[k];
  __syncthreads();
  if (threadIdx.x < LD * 4) {
    const int col = threadIdx.x >> 2, k = threadIdx.x & 3;
    double t = 0.0;
    for (int u = col; u < kBT; u += LD) t += s[u][k];
    partials[((size_t)blockIdx.x * LD + col) * 4 + k] = t;
  }
}

// Per-column p^T q, ||p||^2, ||q||^2 of one row component.
__device__ __forceinline__ void pq_terms(const double2 p, double yr, double yi, double (&acc)[4]) {
  acc[0] += p.x * yr - p.y * yi;
  acc[1] += p.x * yi + p.y * yr;
  acc[2] += p.x * p.x + p.y * p.y;
  acc[3] += yr * yr + yi * yi;
}

// Q = A P on the matrix cores (complex64 matrix, FP32 products per block,
// FP64 sum over blocks), with per-column p^T q.
__global__ void __launch_bounds__(kBT) k_bspmm_mfma(PatternDev pt, const float2* __restrict__ val,
                                                    const double2* __restrict__ P, double2* __restrict__ Q,
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
      const double2* xrow = P + (size_t)3 * c * kLD + lane;
      v4f K1 = {0.f, 0.f, 0.f, 0.f}, K2 = K1, K3 = K1, K4 = K1;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const float2 a = m < 3 ? blk[3 * m + j] : make_float2(0.f, 0.f);
        const double2 xd = xrow[j * kLD];
        const float2 x = make_float2((float)xd.x, (float)xd.y);
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
  store_col_partials<kLD>(acc, partials);
}

// Same product with FP64 vector FMAs (lane = column) on the complex64 matrix
// promoted, or on the complex128 matrix (V = double2).
// The row's column indices (at most 27) come in with one vector load and are
// taken lane by lane with readlane, so each block costs one memory latency
// (its x entries and its matrix values load together) instead of two.
template <typename V>
__global__ void __launch_bounds__(kBT) k_bspmm_vec(PatternDev pt, const V* __restrict__ val,
                                                   const double2* __restrict__ P, double2* __restrict__ Q,
                                                   double* __restrict__ partials, const BatchScalars* sc) {
  if (sc->active == 0) return;
  const int lane = threadIdx.x & 63;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  // XCD x (the workgroups b with b mod 8 = x; the grid is a multiple of 8)
  // takes positions [x nn / 8, (x + 1) nn / 8) of the row order, its waves
  // sweeping them front to back, so one XCD's L2 holds the gathered
  // directions of a compact slab of the mesh.
  const int xcd = blockIdx.x & 7;
  const int wpx = (int)(gridDim.x >> 3) * (kBT / 64);
  const int pend = (int)(((int64_t)pt.nn * (xcd + 1)) >> 3);
  for (int pos = (int)(((int64_t)pt.nn * xcd) >> 3) + (int)(blockIdx.x >> 3) * (kBT / 64) + (threadIdx.x >> 6);
       pos < pend; pos += wpx) {
    const int r = pt.row_order ? uniform_int(pt.row_order[pos]) : pos;
    const int beg = uniform_int(pt.row_ptr[r]);
    const int end = uniform_int(pt.row_ptr[r + 1]);
    const int cl = lane < end - beg ? pt.col_idx[beg + lane] : 0;
    double yr[3] = {0.0, 0.0, 0.0}, yi[3] = {0.0, 0.0, 0.0};
    for (int b = beg; b < end; ++b) {
      const int c = __builtin_amdgcn_readlane(cl, b - beg);
      const V* blk = val + (size_t)b * 9;
      const double2* xrow = P + (size_t)3 * c * kLD + lane;
      const double2 x0 = xrow[0], x1 = xrow[kLD], x2 = xrow[2 * kLD];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double2 a0 = as_f64(blk[3 * i]), a1 = as_f64(blk[3 * i + 1]), a2 = as_f64(blk[3 * i + 2]);
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
  store_col_partials<kLD>(acc, partials);
}

// Narrow SpMM (LD <= 4 columns): one block row per wave in the single-RHS
// mapping; each lane's matrix values multiply the gathered x of every
// column.  The per-column p^T q sums of the output lanes (0, 3, 6) are
// reduced over the wave and then over the workgroup in fixed order.
template <int LD, typename V>
__global__ void __launch_bounds__(kBT) k_bspmm_mc(PatternDev pt, const V* __restrict__ val,
                                                  const double2* __restrict__ P, double2* __restrict__ Q,
                                                  double* __restrict__ partials, const BatchScalars* sc) {
  if (sc->active == 0) return;
  const int lane = threadIdx.x & 63;
  const int e = lane % 9, bo = lane / 9, j = e % 3;
  const bool out_lane = lane == 0 || lane == 3 || lane == 6;
  double acc[LD][4];
#pragma unroll
  for (int c = 0; c < LD; ++c)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[c][k] = 0.0;
  int nwaves;
  for (int r = wave_index(kBT / 64, nwaves); r < pt.nn; r += nwaves) {
    const int beg = uniform_int(pt.row_ptr[r]);
    int nb = uniform_int(pt.row_ptr[r + 1]) - beg;
    if (lane >= 63) nb = 0;
    double2 a[4];
    int32_t cidx[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int b = bo + 7 * kk;
      if (b < nb) {
        a[kk] = as_f64(val[(size_t)(beg + b) * 9 + e]);
        cidx[kk] = pt.col_idx[beg + b];
      }
    }
    double ar[LD], ai[LD];
#pragma unroll
    for (int c = 0; c < LD; ++c) ar[c] = ai[c] = 0.0;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      if (bo + 7 * kk < nb) {
        const double2* xr = P + ((size_t)3 * cidx[kk] + j) * LD;
#pragma unroll
        for (int c = 0; c < LD; ++c) {
          const double2 xv = xr[c];
          ar[c] += a[kk].x * xv.x - a[kk].y * xv.y;
          ai[c] += a[kk].x * xv.y + a[kk].y * xv.x;
        }
      }
    }
    const bool keep = lane < 63 && (lane % 3) == 0;
#pragma unroll
    for (int c = 0; c < LD; ++c) {
      const double r1 = __shfl_down(ar[c], 1, 64), i1 = __shfl_down(ai[c], 1, 64);
      const double r2 = __shfl_down(ar[c], 2, 64), i2 = __shfl_down(ai[c], 2, 64);
      double yr = keep ? ar[c] + r1 + r2 : 0.0;
      double yi = keep ? ai[c] + i1 + i2 : 0.0;
      double t;
      t = __shfl_down(yr, 36, 64); yr += lane + 36 < 64 ? t : 0.0;
      t = __shfl_down(yi, 36, 64); yi += lane + 36 < 64 ? t : 0.0;
      t = __shfl_down(yr, 18, 64); yr += lane + 18 < 64 ? t : 0.0;
      t = __shfl_down(yi, 18, 64); yi += lane + 18 < 64 ? t : 0.0;
      t = __shfl_down(yr, 9, 64); yr += lane + 9 < 64 ? t : 0.0;
      t = __shfl_down(yi, 9, 64); yi += lane + 9 < 64 ? t : 0.0;
      if (out_lane) {
        const size_t idx = (size_t)(3 * r + lane / 3) * LD + c;
        Q[idx] = make_double2(yr, yi);
        const double2 p = P[idx];
        acc[c][0] += p.x * yr - p.y * yi;
        acc[c][1] += p.x * yi + p.y * yr;
        acc[c][2] += p.x * p.x + p.y * p.y;
        acc[c][3] += yr * yr + yi * yi;
      }
    }
  }
  // lanes 0, 3, 6 of each wave -> workgroup partials[block][c][4]
  __shared__ double s[kBT / 64][3][LD][4];
  const int wid = threadIdx.x >> 6;
  if (out_lane)
#pragma unroll
    for (int c = 0; c < LD; ++c)
#pragma unroll
      for (int k = 0; k < 4; ++k) s[wid][lane / 3][c][k] = acc[c][k];
  __syncthreads();
  if (threadIdx.x < LD * 4) {
    const int c = threadIdx.x >> 2, k = threadIdx.x & 3;
    double t = 0.0;
    for (int w = 0; w < kBT / 64; ++w)
      for (int o = 0; o < 3; ++o) t += s[w][o][c][k];
    partials[((size_t)blockIdx.x * LD + c) * 4 + k] = t;
  }
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
template <int LD>
__device__ __forceinline__ void column_total(const double* __restrict__ partials, int nblocks, int col,
                                             double (&tot)[4]) {
  __shared__ double s[kBT][4];
  double v[4] = {0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += kBT)
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] += partials[((size_t)b * LD + col) * 4 + k];
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
template <int LD>
__global__ void __launch_bounds__(kBT) k_bred_alpha(const double* __restrict__ partials, int nblocks, BatchScalars* sc) {
  if (sc->active == 0) return;
  const int col = blockIdx.x;
  double t[4];
  column_total<LD>(partials, nblocks, col, t);
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
template <int LD>
__global__ void __launch_bounds__(kBT) k_bred_beta(const double* __restrict__ partials, int nblocks, BatchScalars* sc) {
  if (sc->active == 0) return;
  const int col = blockIdx.x;
  double t[4];
  column_total<LD>(partials, nblocks, col, t);
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
template <int LD>
__global__ void __launch_bounds__(kBT) k_bupdate(int64_t n, const double2* __restrict__ dinv, double2* __restrict__ X,
                                                 double2* __restrict__ R, const double2* __restrict__ P,
                                                 const double2* __restrict__ Q, double* __restrict__ partials,
                                                 const BatchScalars* sc) {
  if (sc->active == 0) return;
  const int col = threadIdx.x % LD;
  const bool on = sc->done[col] == 0;
  const double ar = sc->alpha[col].x, ai = sc->alpha[col].y;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t rows_per_block = kBT / LD;
  for (int64_t u = (int64_t)blockIdx.x * rows_per_block + threadIdx.x / LD; u < n;
       u += (int64_t)gridDim.x * rows_per_block) {
    if (!on) continue;
    const size_t idx = (size_t)u * LD + col;
    const double2 p = P[idx];
    const double2 q = Q[idx];
    const double2 d = dinv[u];
    double2 x = X[idx];
    double2 r = R[idx];
    x.x += ar * p.x - ai * p.y;
    x.y += ar * p.y + ai * p.x;
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
  store_col_partials<LD>(v, partials);
}

// p = D^-1 r + beta p for running columns, or for the columns with
// only[c] == 1 right after a reliable update.
template <int LD>
__global__ void __launch_bounds__(kBT) k_bpupdate(int64_t n, const double2* __restrict__ dinv,
                                                  const double2* __restrict__ R, double2* __restrict__ P,
                                                  const BatchScalars* sc, const int32_t* __restrict__ only) {
  if (sc->active == 0 && !only) return;
  const int col = threadIdx.x % LD;
  const bool on = only ? only[col] == 1 : sc->done[col] == 0;
  if (!on) return;
  const double br = sc->beta[col].x, bi = sc->beta[col].y;
  const int64_t rows_per_block = kBT / LD;
  for (int64_t u = (int64_t)blockIdx.x * rows_per_block + threadIdx.x / LD; u < n;
       u += (int64_t)gridDim.x * rows_per_block) {
    const size_t idx = (size_t)u * LD + col;
    const double2 d = dinv[u], r = R[idx];
    const double2 p = P[idx];
    const double zr = d.x * r.x - d.y * r.y, zi = d.x * r.y + d.y * r.x;
    P[idx] = make_double2(zr + br * p.x - bi * p.y, zi + br * p.y + bi * p.x);
  }
}

// ------------------------------------------------------------ FP64 parts
// R = B - A X in FP64 for the columns with mask[c] != 0 (all when mask is
// null); per-column ||B - A X||^2 for every column.  Lane l works on column
// l % LD of block row (wave row) * (64 / LD) + l / LD.  Once per reliable
// update, so it favours simplicity over speed.
template <int LD>
__global__ void __launch_bounds__(kBT) k_bresidual64(PatternDev pt, const double2* __restrict__ val,
                                                     const double2* __restrict__ X, const double2* __restrict__ B,
                                                     double2* __restrict__ R, double* __restrict__ partials,
                                                     const int32_t* __restrict__ mask) {
  const int lane = threadIdx.x & 63;
  const int col = lane % LD, slot = lane / LD;
  constexpr int kRowsPerWave = 64 / LD;
  const bool store = mask ? mask[col] != 0 : true;
  double acc = 0.0;
  int nwaves;
  for (int r0 = wave_index(kBT / 64, nwaves) * kRowsPerWave; r0 < pt.nn; r0 += nwaves * kRowsPerWave) {
    const int r = r0 + slot;
    if (r >= pt.nn) continue;
    const int beg = pt.row_ptr[r];
    const int end = pt.row_ptr[r + 1];
    double yr[3] = {0, 0, 0}, yi[3] = {0, 0, 0};
    for (int b = beg; b < end; ++b) {
      const int c = pt.col_idx[b];
      const double2* blk = val + (size_t)b * 9;
      const double2* xrow = X + (size_t)3 * c * LD + col;
      const double2 x0 = xrow[0], x1 = xrow[LD], x2 = xrow[2 * LD];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double2 a0 = blk[3 * i], a1 = blk[3 * i + 1], a2 = blk[3 * i + 2];
        yr[i] += a0.x * x0.x - a0.y * x0.y + a1.x * x1.x - a1.y * x1.y + a2.x * x2.x - a2.y * x2.y;
        yi[i] += a0.x * x0.y + a0.y * x0.x + a1.x * x1.y + a1.y * x1.x + a2.x * x2.y + a2.y * x2.x;
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const size_t idx = (size_t)(3 * r + i) * LD + col;
      const double2 bv = B[idx];
      const double2 rv = make_double2(bv.x - yr[i], bv.y - yi[i]);
      if (store) R[idx] = rv;
      acc += rv.x * rv.x + rv.y * rv.y;
    }
  }
  __shared__ double s[kBT];
  s[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < LD) {
    double t = 0.0;
    for (int u = threadIdx.x; u < kBT; u += LD) t += s[u];
    partials[(size_t)blockIdx.x * LD + threadIdx.x] = t;
  }
}

template <int LD>
__global__ void __launch_bounds__(kBT) k_bred_norm64(const double* __restrict__ partials, int nblocks,
                                                     double* __restrict__ rr64) {
  const int col = blockIdx.x;
  __shared__ double s[kBT];
  double v = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kBT) v += partials[(size_t)b * LD + col];
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
template <int LD>
__global__ void __launch_bounds__(kBT) k_brescale(int64_t n, const double2* __restrict__ R,
                                                  const double2* __restrict__ dinv, double2* __restrict__ P,
                                                  double* __restrict__ partials, const BatchPlan* __restrict__ plan) {
  const int col = threadIdx.x % LD;
  const int act = plan->action[col];
  const bool on = act == 1 || act == 2;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t rows_per_block = kBT / LD;
  if (on) {
    for (int64_t u = (int64_t)blockIdx.x * rows_per_block + threadIdx.x / LD; u < n;
         u += (int64_t)gridDim.x * rows_per_block) {
      const size_t idx = (size_t)u * LD + col;
      const double2 r = R[idx];
      const double2 d = dinv[u];
      const double zr = d.x * r.x - d.y * r.y, zi = d.x * r.y + d.y * r.x;
      if (act == 2) P[idx] = make_double2(zr, zi);
      v[0] += r.x * zr - r.y * zi;
      v[1] += r.x * zi + r.y * zr;
      v[2] += r.x * r.x + r.y * r.y;
      v[3] += zr * zr + zi * zi;
    }
  }
  store_col_partials<LD>(v, partials);
}

template <int LD>
__global__ void __launch_bounds__(kBT) k_bred_rescale(const double* __restrict__ partials, int nblocks,
                                                      BatchScalars* sc, const BatchPlan* __restrict__ plan) {
  const int col = blockIdx.x;
  const int act = plan->action[col];
  if (act != 1 && act != 2) {
    if (threadIdx.x == 0 && act == 3) sc->done[col] = plan->final_state[col];
    return;
  }
  double t[4];
  column_total<LD>(partials, nblocks, col, t);
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

// Minimal-residual step for the columns restarting after a breakdown
// (plan->action == 2): with p = D^-1 r and w = A p in Q, omega = w^H r /
// w^H w (Hermitian products), x += omega p, r -= omega w.  It cannot raise
// ||r|| and moves r off the direction on which the bilinear form of the
// conjugate-orthogonal recurrence vanished, so the restart that follows
// does not break down again at once.
template <int LD>
__global__ void __launch_bounds__(kBT) k_bmr_dots(int64_t n, const double2* __restrict__ R,
                                                  const double2* __restrict__ Q, double* __restrict__ partials,
                                                  const BatchPlan* __restrict__ plan) {
  const int col = threadIdx.x % LD;
  const bool on = plan->action[col] == 2;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t rows_per_block = kBT / LD;
  if (on) {
    for (int64_t u = (int64_t)blockIdx.x * rows_per_block + threadIdx.x / LD; u < n;
         u += (int64_t)gridDim.x * rows_per_block) {
      const size_t idx = (size_t)u * LD + col;
      const double2 w = Q[idx], r = R[idx];
      v[0] += w.x * r.x + w.y * r.y;
      v[1] += w.x * r.y - w.y * r.x;
      v[2] += w.x * w.x + w.y * w.y;
    }
  }
  store_col_partials<LD>(v, partials);
}

template <int LD>
__global__ void __launch_bounds__(kBT) k_bred_mr(const double* __restrict__ partials, int nblocks,
                                                 BatchScalars* sc, const BatchPlan* __restrict__ plan) {
  const int col = blockIdx.x;
  if (plan->action[col] != 2) return;
  double t[4];
  column_total<LD>(partials, nblocks, col, t);
  if (threadIdx.x == 0) sc->alpha[col] = t[2] > 0.0 ? make_double2(t[0] / t[2], t[1] / t[2]) : make_double2(0.0, 0.0);
}

template <int LD>
__global__ void __launch_bounds__(kBT) k_bmr_apply(int64_t n, double2* __restrict__ X, double2* __restrict__ R,
                                                   const double2* __restrict__ P, const double2* __restrict__ Q,
                                                   const BatchScalars* sc, const BatchPlan* __restrict__ plan) {
  const int col = threadIdx.x % LD;
  if (plan->action[col] != 2) return;
  const double wr = sc->alpha[col].x, wi = sc->alpha[col].y;
  const int64_t rows_per_block = kBT / LD;
  for (int64_t u = (int64_t)blockIdx.x * rows_per_block + threadIdx.x / LD; u < n;
       u += (int64_t)gridDim.x * rows_per_block) {
    const size_t idx = (size_t)u * LD + col;
    const double2 p = P[idx], q = Q[idx];
    double2 x = X[idx], r = R[idx];
    x.x += wr * p.x - wi * p.y;
    x.y += wr * p.y + wi * p.x;
    r.x -= wr * q.x - wi * q.y;
    r.y -= wr * q.y + wi * q.x;
    X[idx] = x;
    R[idx] = r;
  }
}

__global__ void k_bcount_active(BatchScalars* sc, int ncols) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int act = 0;
    for (int c = 0; c < ncols; ++c) act += sc->done[c] == 0;
    sc->active = act;
  }
}

__global__ void k_product_scalars(BatchScalars* sc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) sc->active = 1;
}

// [nrhs][n] column-major right-hand sides -> [n][LD] block layout (zero pad).
__global__ void k_to_block(int64_t n, int ld, int nrhs, const double2* __restrict__ b, double2* __restrict__ B) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * ld) return;
  const int64_t u = t / ld;
  const int col = (int)(t % ld);
  B[t] = col < nrhs ? b[(size_t)col * n + u] : make_double2(0.0, 0.0);
}

// [n][LD] block layout -> [nrhs][n]
__global__ void k_from_block(int64_t n, int ld, int nrhs, const double2* __restrict__ X, double2* __restrict__ x) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nrhs) return;
  const int64_t r = t / n;
  const int64_t u = t % n;
  x[t] = X[(size_t)u * ld + r];
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

int batched_vec_blocks(int64_t n, int ld) {
  const int64_t rows_per_block = kBT / ld;
  int64_t b = (n + rows_per_block - 1) / rows_per_block;
  if (b > 2048) b = 2048;
  if (b < 8) b = 8;
  return (int)b;
}

#define FEMH_LD_DISPATCH(ld, CALL) \
  do {                             \
    if ((ld) == 4) {               \
      constexpr int LD = 4;        \
      CALL;                        \
    } else {                       \
      constexpr int LD = 64;       \
      CALL;                        \
    }                              \
  } while (0)

hipError_t bspmm(hipStream_t st, const PatternDev& pt, const float2* val32, const double2* val64, const double2* P,
                 double2* Q, double* partials, const BatchScalars* sc, BatchTile tile) {
  if (tile.kind == 1)  // matrix cores: complex64 matrix only
    hipLaunchKernelGGL(k_bspmm_mfma, dim3(tile.blocks), dim3(kBT), 0, st, pt, val32, P, Q, partials, sc);
  else if (tile.kind == 2 && val64)
    hipLaunchKernelGGL((k_bspmm_mc<4, double2>), dim3(tile.blocks), dim3(kBT), 0, st, pt, val64, P, Q, partials, sc);
  else if (tile.kind == 2)
    hipLaunchKernelGGL((k_bspmm_mc<4, float2>), dim3(tile.blocks), dim3(kBT), 0, st, pt, val32, P, Q, partials, sc);
  else if (val64)
    hipLaunchKernelGGL(k_bspmm_vec<double2>, dim3(tile.blocks), dim3(kBT), 0, st, pt, val64, P, Q, partials, sc);
  else
    hipLaunchKernelGGL(k_bspmm_vec<float2>, dim3(tile.blocks), dim3(kBT), 0, st, pt, val32, P, Q, partials, sc);
  return hipGetLastError();
}

hipError_t bred_alpha(hipStream_t st, const double* partials, int nblocks, int ld, BatchScalars* sc) {
  FEMH_LD_DISPATCH(ld, hipLaunchKernelGGL(k_bred_alpha<LD>, dim3(LD), dim3(kBT), 0, st, partials, nblocks, sc));
  return hipGetLastError();
}

hipError_t bupdate(hipStream_t st, int64_t n, int ld, const double2* dinv, double2* X, double2* R, const double2* P,
                   const double2* Q, double* partials, int blocks, const BatchScalars* sc) {
  FEMH_LD_DISPATCH(ld, hipLaunchKernelGGL(k_bupdate<LD>, dim3(blocks), dim3(kBT), 0, st, n, dinv, X, R, P, Q,
                                          partials, sc));
  return hipGetLastError();
}

hipError_t bred_beta(hipStream_t st, const double* partials, int nblocks, int ld, BatchScalars* sc) {
  FEMH_LD_DISPATCH(ld, hipLaunchKernelGGL(k_bred_beta<LD>, dim3(LD), dim3(kBT), 0, st, partials, nblocks, sc));
  return hipGetLastError();
}

hipError_t bpupdate(hipStream_t st, int64_t n, int ld, const double2* dinv, const double2* R, double2* P, int blocks,
                    const BatchScalars* sc, const int32_t* only) {
  FEMH_LD_DISPATCH(ld, hipLaunchKernelGGL(k_bpupdate<LD>, dim3(blocks), dim3(kBT), 0, st, n, dinv, R, P, sc, only));
  return hipGetLastError();
}

hipError_t bresidual64(hipStream_t st, const PatternDev& pt, int ld, const double2* val, const double2* X,
                       const double2* B, double2* R, double* partials, int blocks, double* rr64,
                       const int32_t* mask) {
  FEMH_LD_DISPATCH(ld, {
    hipLaunchKernelGGL(k_bresidual64<LD>, dim3(blocks), dim3(kBT), 0, st, pt, val, X, B, R, partials, mask);
    hipLaunchKernelGGL(k_bred_norm64<LD>, dim3(LD), dim3(kBT), 0, st, (const double*)partials, blocks, rr64);
  });
  return hipGetLastError();
}

hipError_t brescale(hipStream_t st, int64_t n, int ld, const double2* R, const double2* dinv, double2* P,
                    double* partials, int blocks, BatchScalars* sc, const BatchPlan* plan) {
  FEMH_LD_DISPATCH(ld, {
    hipLaunchKernelGGL(k_brescale<LD>, dim3(blocks), dim3(kBT), 0, st, n, R, dinv, P, partials, plan);
    hipLaunchKernelGGL(k_bred_rescale<LD>, dim3(LD), dim3(kBT), 0, st, (const double*)partials, blocks, sc, plan);
    hipLaunchKernelGGL(k_bcount_active, dim3(1), dim3(64), 0, st, sc, LD);
  });
  return hipGetLastError();
}

hipError_t bmr_step(hipStream_t st, const PatternDev& pt, int64_t n, int ld, const float2* val32,
                    const double2* val64, double2* X, double2* R, const double2* P, double2* Q, double* partials,
                    int blocks, BatchTile tile, const BatchScalars* run_all, BatchScalars* sc,
                    const BatchPlan* plan) {
  hipError_t e = bspmm(st, pt, val32, val64, P, Q, partials, run_all, tile);
  if (e != hipSuccess) return e;
  FEMH_LD_DISPATCH(ld, {
    hipLaunchKernelGGL(k_bmr_dots<LD>, dim3(blocks), dim3(kBT), 0, st, n, R, Q, partials, plan);
    hipLaunchKernelGGL(k_bred_mr<LD>, dim3(LD), dim3(kBT), 0, st, (const double*)partials, blocks, sc, plan);
    hipLaunchKernelGGL(k_bmr_apply<LD>, dim3(blocks), dim3(kBT), 0, st, n, X, R, P, Q, sc, plan);
  });
  return hipGetLastError();
}

hipError_t product_scalars(hipStream_t st, BatchScalars* sc) {
  hipLaunchKernelGGL(k_product_scalars, dim3(1), dim3(64), 0, st, sc);
  return hipGetLastError();
}

hipError_t to_block(hipStream_t st, int64_t n, int ld, int nrhs, const double2* b, double2* B) {
  const int64_t t = n * ld;
  hipLaunchKernelGGL(k_to_block, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, n, ld, nrhs, b, B);
  return hipGetLastError();
}

hipError_t from_block(hipStream_t st, int64_t n, int ld, int nrhs, const double2* X, double2* x) {
  const int64_t t = n * nrhs;
  hipLaunchKernelGGL(k_from_block, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, n, ld, nrhs, X, x);
  return hipGetLastError();
}

}  // namespace k
}  // namespace femh
