// Block incomplete Cholesky preconditioner (sections 3.1.5.2-3.1.5.3).
//
// The unknowns are cut into blocks of B consecutive nodes (3 B unknowns);
// couplings between blocks are dropped, as each of the paper's processors
// keeps only its diagonal block.  Inside a block, eq. (5)'s incomplete
// factor A ~ L L^T (no conjugation: A is complex-symmetric) keeps the lower
// part of A's block pattern: every entry of the 3x3 block of two nodes that
// share an element, the diagonal block's lower triangle included.
//
// L is a scalar CSR matrix [3 Nn rows], columns ascending within a row, the
// diagonal last.  It is built from the block CSR matrix in two
// data-parallel passes (count, then fill after a scan) and factorised in
// place by one thread per block (a block's rows depend on each other in
// order; all blocks run at once), which also stores 1 / l_uu.  U, the
// strict upper part of L^T (the columns of L as rows), is built by a search
// of the block's later rows.
//
// The application z = (L L^T)^-1 r runs one wavefront per block: the
// block's slice of the vector lives in LDS, and eq. (6)'s two substitutions
// run as column sweeps.  Forward (L y = r): for u ascending, y_u = r_u /
// l_uu, then every later entry of column u takes its update y_v -= l_vu y_u,
// one lane per entry (distinct v, so no reduction and no conflict).  Back
// (L^T z = y): for u descending, z_u = y_u / l_uu, then y_v -= l_uv z_u over
// row u of L.  The rows' entries are staged into LDS in chunks of up to 64
// rows, so each step reads only LDS, and a step needs no barrier (one
// wavefront, whose LDS operations complete in order).
#include "internal.h"

namespace femh {
namespace {

constexpr int kFactorThreads = 64;
constexpr int kChunkRows = 64;  // staged rows per chunk (one per lane)

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a / b, scaled so that |b|^2 neither overflows nor underflows
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double s = fmax(fabs(b.x), fabs(b.y));
  const double br = b.x / s, bi = b.y / s;
  const double d = br * br + bi * bi;
  return make_double2((a.x * br + a.y * bi) / (d * s), (a.y * br - a.x * bi) / (d * s));
}
// principal square root (non-negative real part)
__device__ __forceinline__ double2 csqrt(double2 z) {
  const double r = hypot(z.x, z.y);
  if (r == 0.0) return make_double2(0.0, 0.0);
  if (z.x >= 0.0) {
    const double t = sqrt(0.5 * (r + z.x));
    return make_double2(t, z.y / (2.0 * t));
  }
  const double t = sqrt(0.5 * (r - z.x));
  return make_double2(fabs(z.y) / (2.0 * t), copysign(t, z.y));
}

// Entries of scalar row u = 3 a + i of L: the blocks (a, c) of the block
// row with c in a's block and c <= a; 3 columns for c < a, i + 1 for c = a.
__global__ void k_bic_count(int32_t nn, int32_t nodes_per_block, const int32_t* __restrict__ row_ptr,
                            const int32_t* __restrict__ col_idx, int32_t* __restrict__ counts) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= 3 * (int64_t)nn) return;
  const int32_t a = (int32_t)(u / 3), i = (int32_t)(u % 3);
  const int32_t blk = a / nodes_per_block;
  int32_t cnt = 0;
  for (int32_t b = row_ptr[a]; b < row_ptr[a + 1]; ++b) {
    const int32_t c = col_idx[b];
    if (c > a) break;
    if (c / nodes_per_block == blk) cnt += c < a ? 3 : i + 1;
  }
  counts[u] = cnt;
}

// Columns and A's values of L's rows, at the offsets of the scan.
__global__ void k_bic_fill(int32_t nn, int32_t nodes_per_block, const int32_t* __restrict__ row_ptr,
                           const int32_t* __restrict__ col_idx, const double2* __restrict__ val,
                           const int32_t* __restrict__ lrp, int32_t* __restrict__ lcol,
                           double2* __restrict__ lval) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= 3 * (int64_t)nn) return;
  const int32_t a = (int32_t)(u / 3), i = (int32_t)(u % 3);
  const int32_t blk = a / nodes_per_block;
  int32_t k = lrp[u];
  for (int32_t b = row_ptr[a]; b < row_ptr[a + 1]; ++b) {
    const int32_t c = col_idx[b];
    if (c > a) break;
    if (c / nodes_per_block != blk) continue;
    const int jn = c < a ? 3 : i + 1;
    for (int j = 0; j < jn; ++j) {
      lcol[k] = 3 * c + j;
      lval[k] = val[(size_t)b * 9 + 3 * i + j];
      ++k;
    }
  }
}

// In-place IC(0) of one block per thread, row by row: for each entry
// (u, v < u) in ascending v, l_uv = (a_uv - sum_w l_uw l_vw) / l_vv over the
// columns w < v present in both rows (a merge of two sorted rows); then
// l_uu = sqrt(a_uu - sum_w l_uw^2) and dinv_u = 1 / l_uu.  A pivot that is
// zero or not finite sets *bad.
__global__ void __launch_bounds__(kFactorThreads) k_bic_factor(int64_t n, int32_t rows_per_block, int32_t nblk,
                                                               const int32_t* __restrict__ lrp,
                                                               const int32_t* __restrict__ lcol,
                                                               double2* __restrict__ lval, double2* __restrict__ ldinv,
                                                               int32_t* bad) {
  const int32_t blk = blockIdx.x * blockDim.x + threadIdx.x;
  if (blk >= nblk) return;
  const int64_t u0 = (int64_t)blk * rows_per_block;
  const int64_t u1 = u0 + rows_per_block < n ? u0 + rows_per_block : n;
  int32_t failed = 0;
  for (int64_t u = u0; u < u1; ++u) {
    const int32_t rs = lrp[u], re = lrp[u + 1];
    double2 d = lval[re - 1];
    for (int32_t e = rs; e < re - 1; ++e) {
      const int32_t v = lcol[e];
      const int32_t vs = lrp[v], ve = lrp[v + 1];
      double2 s = lval[e];
      int32_t x = rs, y = vs;
      while (x < e && y < ve - 1) {
        const int32_t cx = lcol[x], cy = lcol[y];
        if (cx == cy) {
          const double2 t = cmul(lval[x], lval[y]);
          s.x -= t.x;
          s.y -= t.y;
          ++x;
          ++y;
        } else if (cx < cy) {
          ++x;
        } else {
          ++y;
        }
      }
      const double2 l = cdiv(s, lval[ve - 1]);
      lval[e] = l;
      const double2 t = cmul(l, l);
      d.x -= t.x;
      d.y -= t.y;
    }
    const double2 p = csqrt(d);
    if (!(isfinite(p.x) && isfinite(p.y)) || (p.x == 0.0 && p.y == 0.0)) failed = 1;
    lval[re - 1] = p;
    ldinv[u] = failed ? make_double2(0.0, 0.0) : cdiv(make_double2(1.0, 0.0), p);
  }
  if (failed) *bad = 1;
}

// U = strict upper part of L^T: row v holds the rows u > v of v's block whose
// L row has column v (found by bisection of the ascending columns), with
// l_uv.  counts non-null: write the entry counts; else fill at urp's offsets.
__global__ void k_bic_upper(int64_t n, int32_t rows_per_block, const int32_t* __restrict__ lrp,
                            const int32_t* __restrict__ lcol, const double2* __restrict__ lval,
                            int32_t* __restrict__ counts, const int32_t* __restrict__ urp,
                            int32_t* __restrict__ ucol, double2* __restrict__ uval) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int64_t u1 = (v / rows_per_block + 1) * (int64_t)rows_per_block < n
                         ? (v / rows_per_block + 1) * (int64_t)rows_per_block
                         : n;
  int32_t k = counts ? 0 : urp[v];
  for (int64_t u = v + 1; u < u1; ++u) {
    int32_t lo = lrp[u], hi = lrp[u + 1] - 1;  // off-diagonal entries [lo, hi)
    const int32_t end = hi;
    while (lo < hi) {
      const int32_t mid = (lo + hi) >> 1;
      if (lcol[mid] < v) lo = mid + 1;
      else hi = mid;
    }
    if (lo < end && lcol[lo] == v) {
      if (!counts) {
        ucol[k] = (int32_t)u;
        uval[k] = lval[lo];
      }
      ++k;
    }
  }
  if (counts) counts[v] = k;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// A chunk of staged rows in LDS (layout from the launch's dynamic LDS): up
// to kChunkRows rows and cap entries, where cap is at least the factor's
// longest row, so every chunk advances.  Columns are block-relative.
struct Chunk {
  double2* val;   // [cap]
  double2* dinv;  // [kChunkRows] 1 / l_uu of the chunk's rows
  int32_t* col;   // [cap]
  int32_t* rp;    // [kChunkRows + 1] row starts relative to the chunk
};

__device__ __forceinline__ void stage_rows(const Chunk& ch, int64_t u0, int32_t c0, int32_t cnt,
                                           const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                           const double2* __restrict__ val, const double2* __restrict__ dinv,
                                           int lane) {
  const int32_t base = rp[u0 + c0];
  if (lane <= cnt) ch.rp[lane] = rp[u0 + c0 + lane] - base;
  if (lane == 0 && cnt == kChunkRows) ch.rp[kChunkRows] = rp[u0 + c0 + kChunkRows] - base;
  if (lane < cnt) ch.dinv[lane] = dinv[u0 + c0 + lane];
  const int32_t ne = rp[u0 + c0 + cnt] - base;
  for (int32_t t = lane; t < ne; t += 64) {
    ch.val[t] = val[base + t];
    ch.col[t] = (int32_t)(col[base + t] - u0);
  }
}

// The column steps of one staged chunk, ascending (forward sweep, U rows) or
// descending (back sweep, L rows without their diagonal).  Step k: y_k *=
// 1 / l_kk, then y_v -= w y_k over the row's entries (v, w), one lane per
// entry; a lane without an entry updates the spare slot y[spare] with
// weight 0, so every lane issues the same two reads and one write, with no
// branch, and the two reads are in flight together.  kLong: some row of
// the chunk has more than 64 entries, and lanes loop over the rest.  Lane t
// keeps row t's bounds in registers, read back per step with readlane; each
// lane's entry of the next row is read from LDS a step ahead (at a clamped
// index, then selected).  One wavefront owns the block and its LDS
// operations complete in issue order, so a step sees every earlier step's
// updates without a barrier.
template <bool kBack, bool kLong>
__device__ __forceinline__ void sweep_chunk(double2* y, int32_t spare, const Chunk& ch, int32_t cap, int32_t c0,
                                            int32_t cnt, int lane) {
  const int32_t my_s = lane < cnt ? ch.rp[lane] : 0;
  const int32_t my_e = lane < cnt ? ch.rp[lane + 1] - (kBack ? 1 : 0) : 0;
  int32_t k = kBack ? cnt - 1 : 0;
  int32_t rs = __builtin_amdgcn_readlane(my_s, k), re = __builtin_amdgcn_readlane(my_e, k);
  auto fetch = [&](int32_t& v, double2& w) {
    const int32_t i = min(rs + lane, cap - 1);
    const bool has = rs + lane < re;
    const int32_t c = ch.col[i];
    const double2 x = ch.val[i];
    v = has ? c : spare;
    w = has ? x : make_double2(0.0, 0.0);
  };
  int32_t v;
  double2 w;
  fetch(v, w);
  double2 d = ch.dinv[k];
  for (int32_t step = 0; step < cnt; ++step) {
    const double2 yc = y[c0 + k];
    double2 yv = y[v];
    const double2 yk = cmul(yc, d);
    const double2 t = cmul(w, yk);
    yv.x -= t.x;
    yv.y -= t.y;
    y[v] = yv;
    if (kLong) {
      for (int32_t x = rs + 64 + lane; x < re; x += 64) {
        const int32_t vx = ch.col[x];
        const double2 tx = cmul(ch.val[x], yk);
        double2 yx = y[vx];
        yx.x -= tx.x;
        yx.y -= tx.y;
        y[vx] = yx;
      }
    }
    y[c0 + k] = yk;  // every lane stores the same value
    if (step + 1 < cnt) {
      k += kBack ? -1 : 1;
      rs = __builtin_amdgcn_readlane(my_s, k);
      re = __builtin_amdgcn_readlane(my_e, k);
      fetch(v, w);
      d = ch.dinv[k];
    }
  }
}

template <bool kBack>
__device__ __forceinline__ void sweep(double2* y, int32_t spare, const Chunk& ch, int32_t cap, int32_t c0,
                                      int32_t cnt, int lane) {
  const int32_t len = lane < cnt ? ch.rp[lane + 1] - ch.rp[lane] : 0;
  if (__ballot(len > 64)) sweep_chunk<kBack, true>(y, spare, ch, cap, c0, cnt, lane);
  else sweep_chunk<kBack, false>(y, spare, ch, cap, c0, cnt, lane);
}

// z = (L L^T)^-1 r for block blockIdx.x.  Dynamic LDS (bic_apply_lds): the
// block's slice of the vector (rows_per_block complex) and a spare slot,
// then one chunk of cap entries.  The block's r^T z (re, im), ||r||^2 and
// ||z||^2 go to stage[block][4] (k_bic_sum adds them up).  Returns at once
// when the recurrence has stopped (no workgroup of this launch writes the
// flag).
__global__ void __launch_bounds__(64) k_bic_apply(int64_t n, int32_t rows_per_block, int32_t cap,
                                                  const int32_t* __restrict__ lrp, const int32_t* __restrict__ lcol,
                                                  const double2* __restrict__ lval, const int32_t* __restrict__ urp,
                                                  const int32_t* __restrict__ ucol, const double2* __restrict__ uval,
                                                  const double2* __restrict__ ldinv, const double2* __restrict__ r,
                                                  double2* __restrict__ z, double* __restrict__ stage,
                                                  const CocgScalars* sc) {
  if (sc && __builtin_amdgcn_readfirstlane(sc->done)) return;
  extern __shared__ double2 lds[];
  double2* y = lds;
  Chunk ch;
  ch.val = lds + rows_per_block + 1;
  ch.dinv = ch.val + cap;
  ch.col = reinterpret_cast<int32_t*>(ch.dinv + kChunkRows);
  ch.rp = ch.col + cap;
  const int lane = threadIdx.x;
  const int64_t u0 = (int64_t)blockIdx.x * rows_per_block;
  const int32_t m = (int32_t)(u0 + rows_per_block < n ? rows_per_block : n - u0);
  for (int32_t t = lane; t < m; t += 64) y[t] = r[u0 + t];
  if (lane == 0) y[rows_per_block] = make_double2(0.0, 0.0);
  __syncthreads();
  // forward sweep over the columns of L (rows of U), ascending
  for (int32_t c0 = 0; c0 < m;) {
    const int32_t base = urp[u0 + c0];
    const bool fits = c0 + lane + 1 <= m && urp[u0 + c0 + lane + 1] - base <= cap;
    const int32_t cnt = (int32_t)__popcll(__ballot(fits));
    __syncthreads();
    stage_rows(ch, u0, c0, cnt, urp, ucol, uval, ldinv, lane);
    __syncthreads();
    sweep<false>(y, rows_per_block, ch, cap, c0, cnt, lane);
    c0 += cnt;
  }
  // back sweep over the rows of L (diagonal last, not used), descending
  for (int32_t c1 = m; c1 > 0;) {
    const int32_t top = lrp[u0 + c1];
    const bool fits = c1 - 1 - lane >= 0 && top - lrp[u0 + c1 - 1 - lane] <= cap;
    const int32_t cnt = (int32_t)__popcll(__ballot(fits));
    const int32_t c0 = c1 - cnt;
    __syncthreads();
    stage_rows(ch, u0, c0, cnt, lrp, lcol, lval, ldinv, lane);
    __syncthreads();
    sweep<true>(y, rows_per_block, ch, cap, c0, cnt, lane);
    c1 = c0;
  }
  __syncthreads();
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int32_t t = lane; t < m; t += 64) {
    const double2 zt = y[t], rt = r[u0 + t];
    z[u0 + t] = zt;
    acc[0] += rt.x * zt.x - rt.y * zt.y;
    acc[1] += rt.x * zt.y + rt.y * zt.x;
    acc[2] += rt.x * rt.x + rt.y * rt.y;
    acc[3] += zt.x * zt.x + zt.y * zt.y;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] = wave_sum(acc[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) stage[(size_t)blockIdx.x * 4 + k] = acc[k];
  }
}

// The application's per-block sums, added in a fixed order: workgroup g
// sums blocks [g per, (g + 1) per) (thread t every 256th, then a tree), and
// the last workgroup to finish adds the workgroup totals in order into
// out[0..3].  gsum: 4 doubles per workgroup; ticket: zero, and left zero.
constexpr int kSumThreads = 256;
constexpr int kSumGroups = 64;
__global__ void __launch_bounds__(kSumThreads) k_bic_sum(int32_t nblk, int32_t per, const double* __restrict__ stage,
                                                         double* gsum, uint32_t* ticket, double* __restrict__ out,
                                                         const CocgScalars* sc) {
  if (sc && __builtin_amdgcn_readfirstlane(sc->done)) return;
  __shared__ double s[4][kSumThreads];
  __shared__ int s_last;
  const int32_t b0 = blockIdx.x * per;
  const int32_t b1 = b0 + per < nblk ? b0 + per : nblk;
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  for (int32_t b = b0 + threadIdx.x; b < b1; b += kSumThreads)
#pragma unroll
    for (int k = 0; k < 4; ++k) t[k] += stage[(size_t)b * 4 + k];
#pragma unroll
  for (int k = 0; k < 4; ++k) s[k][threadIdx.x] = t[k];
  __syncthreads();
  for (int w = kSumThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < 4; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
      __hip_atomic_store(&gsum[(size_t)blockIdx.x * 4 + k], s[k][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    s_last = atomicAdd(ticket, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last || threadIdx.x != 0) return;
  __threadfence();
  double tot[4] = {0.0, 0.0, 0.0, 0.0};
  for (int32_t g = 0; g < (int32_t)gridDim.x; ++g)
#pragma unroll
    for (int k = 0; k < 4; ++k)
      tot[k] += __hip_atomic_load(&gsum[(size_t)g * 4 + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
  for (int k = 0; k < 4; ++k) out[k] = tot[k];
  *ticket = 0u;  // ready for the next launch (the kernel boundary orders it)
}

// Segment start after an application z = M^-1 r whose totals are in
// sums[0..3]: p = z; the last workgroup to finish its copy records
// rho = r^T z, ||r||^2 and the start verdict (converged / breakdown) in slot
// par.  Every workgroup reads the stop flag at entry, before it takes its
// ticket, so the flag is written only after all of those reads.
__global__ void __launch_bounds__(256) k_bic_init(int64_t n, const double2* __restrict__ zin,
                                                  double2* __restrict__ p, CocgScalars* sc,
                                                  const double* __restrict__ sums, int par) {
  if (sc->done) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = zin[i];
  __shared__ int s_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    s_last = atomicAdd(&sc->ticket[1], 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (s_last && threadIdx.x == 0) {
    __threadfence();
    sc->ticket[1] = 0u;  // ready for the next launch (the kernel boundary orders it)
    const double2 rho = make_double2(sums[0], sums[1]);
    const double rr = sums[2], zz = sums[3];
    sc->rho[par] = rho;
    sc->rr = rr;
    sc->rr_max[par] = rr;
    sc->iters[par] = sc->iters_out;
    if (sc->bb <= 0.0) sc->bb = rr;
    if (rr <= sc->tol2 * sc->bb) sc->done = 1;
    else if (rho.x * rho.x + rho.y * rho.y <= sc->bd_tol * sc->bd_tol * rr * zz) sc->done = 3;
    if (sc->done) sc->stop_par = par;
  }
}

}  // namespace

namespace k {

hipError_t bic_pattern_count(hipStream_t st, const PatternDev& p, int32_t nodes_per_block, int32_t* counts) {
  const int64_t rows = 3 * (int64_t)p.nn;
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bic_count, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, p.nn, nodes_per_block,
                     p.row_ptr, p.col_idx, counts);
  return hipGetLastError();
}

hipError_t bic_pattern_fill(hipStream_t st, const PatternDev& p, int32_t nodes_per_block, const double2* val,
                            const int32_t* lrp, int32_t* lcol, double2* lval) {
  const int64_t rows = 3 * (int64_t)p.nn;
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bic_fill, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, p.nn, nodes_per_block,
                     p.row_ptr, p.col_idx, val, lrp, lcol, lval);
  return hipGetLastError();
}

hipError_t bic_factor(hipStream_t st, int64_t n, int32_t rows_per_block, int32_t nblk, const int32_t* lrp,
                      const int32_t* lcol, double2* lval, double2* ldinv, int32_t* bad) {
  if (nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bic_factor, dim3((unsigned)((nblk + kFactorThreads - 1) / kFactorThreads)),
                     dim3(kFactorThreads), 0, st, n, rows_per_block, nblk, lrp, lcol, lval, ldinv, bad);
  return hipGetLastError();
}

hipError_t bic_upper(hipStream_t st, int64_t n, int32_t rows_per_block, const int32_t* lrp, const int32_t* lcol,
                     const double2* lval, int32_t* counts, const int32_t* urp, int32_t* ucol, double2* uval) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bic_upper, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, rows_per_block, lrp, lcol,
                     lval, counts, urp, ucol, uval);
  return hipGetLastError();
}

size_t bic_apply_lds(int32_t rows_per_block, int32_t cap) {
  return sizeof(double2) * ((size_t)rows_per_block + 1 + (size_t)cap + kChunkRows) +
         sizeof(int32_t) * ((size_t)cap + kChunkRows + 1);
}

size_t bic_stage_doubles(int32_t nblk) { return 4 * (size_t)nblk + 4 * (size_t)kSumGroups; }

hipError_t bic_apply(hipStream_t st, const BicFactorDev& f, const double2* r, double2* z, double* stage,
                     uint32_t* ticket, double* out, const CocgScalars* sc) {
  if (f.nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bic_apply, dim3((unsigned)f.nblk), dim3(64), bic_apply_lds(f.rows_per_block, f.chunk_cap),
                     st, f.n, f.rows_per_block, f.chunk_cap, f.lrp, f.lcol, f.lval, f.urp, f.ucol, f.uval, f.ldinv, r,
                     z, stage, sc);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // at least 256 blocks per summing workgroup, at most kSumGroups workgroups
  int32_t groups = (f.nblk + kSumThreads - 1) / kSumThreads;
  if (groups > kSumGroups) groups = kSumGroups;
  const int32_t per = (f.nblk + groups - 1) / groups;
  hipLaunchKernelGGL(k_bic_sum, dim3((unsigned)groups), dim3(kSumThreads), 0, st, f.nblk, per, stage,
                     stage + 4 * (size_t)f.nblk, ticket, out, sc);
  return hipGetLastError();
}

hipError_t bic_init(hipStream_t st, int64_t n, const double2* z, double2* p, CocgScalars* sc, const double* sums,
                    int par) {
  const int64_t g = (n + 255) / 256;
  hipLaunchKernelGGL(k_bic_init, dim3((unsigned)(g < 1024 ? (g > 0 ? g : 1) : 1024)), dim3(256), 0, st, n, z, p, sc,
                     sums, par);
  return hipGetLastError();
}

}  // namespace k
}  // namespace femh
