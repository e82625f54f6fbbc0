// Krylov kernels: block-CSR SpMV of the 3x3-block complex matrix (complex128,
// or complex64 with FP32 accumulation), the fused steps of conjugate
// gradients read for a complex-symmetric matrix (COCG: unconjugated bilinear
// form r^T z, Hermitian norm ||r|| for stopping) with diagonal
// preconditioning (section 3.1.5.1), the FP64 true residual and the
// iterative-refinement update.
//
// SpMV mapping.  One wavefront owns one block row at a time.  The row's
// values are a contiguous run of 9 * nb complex numbers (nb <= 27 blocks on
// a hexahedral mesh).  Lane l < 63 always handles entry e = l % 9 of blocks
// l / 9, l / 9 + 7, l / 9 + 14, l / 9 + 21: the wave reads the run in steps
// of 63 consecutive complex values (fully coalesced), every lane keeps a
// fixed (row component i, column component j) so it needs one accumulator,
// and x is gathered as x[3 col + j].  Two shuffle stages (over j, then over
// the 7 block offsets) leave y_i in lane 3 i.  Rows are dealt to waves so
// that the 8 XCDs (workgroups are dispatched round-robin over them) each
// sweep a contiguous window of rows at a time, keeping the x gathers inside
// one L2.
//
// Reductions are deterministic and the iteration kernels use no atomics and
// no device-scope fences: each workgroup writes a partial sum, and the next
// kernel's workgroups each re-reduce all partials in one fixed order (the
// totals are bit-identical everywhere).  Once-per-segment kernels (start,
// reliable update, true residual) let the last workgroup to finish (a
// device-scope ticket) reduce instead.  No floating-point atomics.
#include "internal.h"

namespace femh {
namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kBlock = 64 * kWavesPerBlock;
// entries per thread and grid sweep in the COCG update kernels
constexpr int kPerThread = 2;

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double2 ld_stream(const double2* p) {
  d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 ld_stream(const float2* p) {
  f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(p));
  return make_float2(v.x, v.y);
}

template <typename R> struct Cx;
template <> struct Cx<double> { using T = double2; };
template <> struct Cx<float> { using T = float2; };

template <typename C> __device__ __forceinline__ C mk(double re, double im);
template <> __device__ __forceinline__ double2 mk<double2>(double re, double im) { return make_double2(re, im); }
template <> __device__ __forceinline__ float2 mk<float2>(double re, double im) { return make_float2((float)re, (float)im); }

template <typename R>
__device__ __forceinline__ R shfl_down_z(R v, int off, int lane) {
  R s = __shfl_down(v, off, 64);
  return (lane + off < 64) ? s : R(0);
}

// y_i of NR block rows in lanes 0, 3, 6 (see file comment).  The rows'
// load chains are interleaved so a wave keeps NR rows of loads in flight.
// rows[] are wave-uniform; rows >= nn contribute nothing.
// VC is the stored value type (complex64 values are promoted to R in the
// product when the vectors are complex128).
// With kHalf the values are the symmetric half store: hpos[k] of block slot
// k is the stored block's index, or -(index + 1) when the slot's block is
// the transpose of a stored one (its entry (i, j) is stored entry (j, i)).
template <typename R, int NR, typename VC = typename Cx<R>::T, bool kHalf = false>
__device__ __forceinline__ void rows_product(const PatternDev& p, const VC* __restrict__ val,
                                             const typename Cx<R>::T* __restrict__ x, const int32_t (&rows)[NR],
                                             int lane, R (&yr)[NR], R (&yi)[NR],
                                             const int32_t* __restrict__ hpos = nullptr) {
  using C = typename Cx<R>::T;
  const int e = lane % 9;
  const int bo = lane / 9;
  const int j = e % 3;
  int32_t beg[NR], nb[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    if (rows[k] < p.nn) {
      beg[k] = p.row_ptr[rows[k]];
      nb[k] = p.row_ptr[rows[k] + 1] - beg[k];
    } else {
      beg[k] = 0;
      nb[k] = 0;
    }
    if (lane >= 63) nb[k] = 0;
  }
  VC a[NR][4];
  int32_t c[NR][4];
#pragma unroll
  for (int k = 0; k < NR; ++k)
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int b = bo + 7 * kk;
      if (b < nb[k]) {
        if (kHalf) {
          const int32_t hp = hpos[beg[k] + b];
          const bool tr = hp < 0;
          const size_t q = tr ? (size_t)(-(hp + 1)) : (size_t)hp;
          a[k][kk] = ld_stream(val + q * 9 + (tr ? 3 * (e % 3) + e / 3 : e));
        } else {
          a[k][kk] = ld_stream(val + (size_t)(beg[k] + b) * 9 + e);
        }
        c[k][kk] = p.col_idx[beg[k] + b];
      }
    }
  R ar[NR], ai[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    ar[k] = R(0);
    ai[k] = R(0);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int b = bo + 7 * kk;
      if (b < nb[k]) {
        const C xv = x[3 * (size_t)c[k][kk] + j];
        const R vr = (R)a[k][kk].x, vi = (R)a[k][kk].y;
        ar[k] += vr * xv.x - vi * xv.y;
        ai[k] += vr * xv.y + vi * xv.x;
      }
    }
  }
  const bool keep = lane < 63 && (lane % 3) == 0;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    // stage 1: lanes with j = 0 collect j = 1, 2 of the same (block, i)
    const R r1 = __shfl_down(ar[k], 1, 64), i1 = __shfl_down(ai[k], 1, 64);
    const R r2 = __shfl_down(ar[k], 2, 64), i2 = __shfl_down(ai[k], 2, 64);
    ar[k] = keep ? ar[k] + r1 + r2 : R(0);
    ai[k] = keep ? ai[k] + i1 + i2 : R(0);
    // stage 2: sum the 7 block offsets (lanes 9 bo + 3 i) into lanes 3 i
    ar[k] += shfl_down_z(ar[k], 36, lane);
    ai[k] += shfl_down_z(ai[k], 36, lane);
    ar[k] += shfl_down_z(ar[k], 18, lane);
    ai[k] += shfl_down_z(ai[k], 18, lane);
    ar[k] += shfl_down_z(ar[k], 9, lane);
    ai[k] += shfl_down_z(ai[k], 9, lane);
    yr[k] = ar[k];
    yi[k] = ai[k];
  }
}

__device__ __forceinline__ int wave_row_start(int& nwaves) {
  const int wib = threadIdx.x >> 6;
  const int xcd = blockIdx.x & 7;
  const int loc = blockIdx.x >> 3;
  const int per_xcd = gridDim.x >> 3;
  nwaves = gridDim.x * kWavesPerBlock;
  return __builtin_amdgcn_readfirstlane((xcd * per_xcd + loc) * kWavesPerBlock + wib);
}

constexpr int kRowsPerWave = 1;  // rows a wave keeps in flight (2 costs occupancy: measured slower)

// y = A x from the symmetric half store (see rows_product).
template <typename R, typename VC = typename Cx<R>::T>
__global__ void __launch_bounds__(kBlock) k_spmv_half(PatternDev p, const VC* __restrict__ hval,
                                                      const int32_t* __restrict__ hpos,
                                                      const typename Cx<R>::T* __restrict__ x,
                                                      typename Cx<R>::T* __restrict__ y) {
  using C = typename Cx<R>::T;
  const int lane = threadIdx.x & 63;
  int nwaves;
  const int w = wave_row_start(nwaves);
  for (int32_t r0 = w; r0 < p.nn; r0 += nwaves) {
    int32_t rows[1] = {r0};
    R yr[1], yi[1];
    rows_product<R, 1, VC, true>(p, hval, x, rows, lane, yr, yi, hpos);
    if (lane == 0 || lane == 3 || lane == 6) {
      C o;
      o.x = yr[0];
      o.y = yi[0];
      y[3 * (size_t)r0 + lane / 3] = o;
    }
  }
}

// Copy the stored (lower, column <= row) blocks into the half store.
__global__ void k_gather_half(int64_t nnzb, const int32_t* __restrict__ hpos, const double2* __restrict__ val,
                              double2* __restrict__ hval) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nnzb * 9) return;
  const int64_t q = t / 9;
  const int32_t hp = hpos[q];
  if (hp < 0) return;
  hval[(int64_t)hp * 9 + t % 9] = val[t];
}

template <typename R, typename VC = typename Cx<R>::T>
__global__ void __launch_bounds__(kBlock) k_spmv(PatternDev p, const VC* __restrict__ val,
                                                 const typename Cx<R>::T* __restrict__ x,
                                                 typename Cx<R>::T* __restrict__ y) {
  using C = typename Cx<R>::T;
  const int lane = threadIdx.x & 63;
  int nwaves;
  const int w = wave_row_start(nwaves);
  for (int32_t r0 = w; r0 < p.nn; r0 += kRowsPerWave * nwaves) {
    int32_t rows[kRowsPerWave];
#pragma unroll
    for (int k = 0; k < kRowsPerWave; ++k) rows[k] = r0 + k * nwaves;
    R yr[kRowsPerWave], yi[kRowsPerWave];
    rows_product<R, kRowsPerWave, VC>(p, val, x, rows, lane, yr, yi);
    if (lane == 0 || lane == 3 || lane == 6) {
#pragma unroll
      for (int k = 0; k < kRowsPerWave; ++k)
        if (rows[k] < p.nn) {
          C o;
          o.x = yr[k];
          o.y = yi[k];
          y[3 * (size_t)rows[k] + lane / 3] = o;
        }
    }
  }
}

// ------------------------------------------------------ block reductions
// Sum NV values of type R over the workgroup; result valid in thread 0.
template <typename R, int NV>
__device__ __forceinline__ void block_sum(R (&v)[NV]) {
  __shared__ R s[kBlock / 64][NV > 0 ? NV : 1];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] += __shfl_xor(v[i], off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) s[wid][i] = v[i];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      R t = s[0][i];
      for (int w = 1; w < kBlock / 64; ++w) t += s[w][i];
      v[i] = t;
    }
  }
  __syncthreads();
}

// Workgroup sum of eight values, every thread returning with all eight
// totals.  Within a wave the sums are a reduce-scatter: at lane distance 32
// each lane keeps half of the values and adds its partner's copy of that
// half, then a quarter at 16 and one value at 8, so after distances 4, 2, 1
// lane l holds the wave total of value l >> 3 (10 cross-lane moves for all
// eight values, against 6 per value for a butterfly on each).  The order of
// additions depends on lane and wave indices only, so every workgroup forms
// bit-identical totals from identical inputs.
__device__ __forceinline__ void block_sum8(double (&v)[8]) {
  __shared__ double s_w[kBlock / 64][8];
  __shared__ double s_t[8];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const bool h32 = lane & 32, h16 = lane & 16, h8 = lane & 8;
  double a[4], c[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double give = h32 ? v[i] : v[i + 4];
    const double keep = h32 ? v[i + 4] : v[i];
    a[i] = keep + __shfl_xor(give, 32, 64);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double give = h16 ? a[i] : a[i + 2];
    const double keep = h16 ? a[i + 2] : a[i];
    c[i] = keep + __shfl_xor(give, 16, 64);
  }
  double e = (h8 ? c[1] : c[0]) + __shfl_xor(h8 ? c[0] : c[1], 8, 64);
  e += __shfl_xor(e, 4, 64);
  e += __shfl_xor(e, 2, 64);
  e += __shfl_xor(e, 1, 64);
  if ((lane & 7) == 0) s_w[wid][lane >> 3] = e;
  __syncthreads();
  if (threadIdx.x < 8) {
    double t = s_w[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < kBlock / 64; ++w) t += s_w[w][threadIdx.x];
    s_t[threadIdx.x] = t;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = s_t[i];
}

// The same for four values: at lane distance 32 each lane keeps two, at 16
// one, so after distances 8, 4, 2, 1 lane l holds the wave total of value
// (l >> 4) & 3 (7 cross-lane moves, against 24).
__device__ __forceinline__ void block_sum4(double (&v)[4]) {
  __shared__ double s_w[kBlock / 64][4];
  __shared__ double s_t[4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const bool h32 = lane & 32, h16 = lane & 16;
  double a[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double give = h32 ? v[i] : v[i + 2];
    const double keep = h32 ? v[i + 2] : v[i];
    a[i] = keep + __shfl_xor(give, 32, 64);
  }
  double e = (h16 ? a[1] : a[0]) + __shfl_xor(h16 ? a[0] : a[1], 16, 64);
  e += __shfl_xor(e, 8, 64);
  e += __shfl_xor(e, 4, 64);
  e += __shfl_xor(e, 2, 64);
  e += __shfl_xor(e, 1, 64);
  if ((lane & 15) == 0) s_w[wid][lane >> 4] = e;
  __syncthreads();
  if (threadIdx.x < 4) {
    double t = s_w[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < kBlock / 64; ++w) t += s_w[w][threadIdx.x];
    s_t[threadIdx.x] = t;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = s_t[i];
}

// The stop flag as one decision for the whole workgroup.  In the update
// kernels workgroup 0 records the step's verdict in the flag while the other
// workgroups of the same launch may still be reading it, so a wave-by-wave
// test could split a workgroup: the waves that stay would then sum the LDS
// slots of the waves that left (block_sum4/8) and update their entries with
// those garbage totals.  Each wave reads the flag early (its latency hides
// under the operand loads that follow), and the workgroup exits if any of
// its waves saw it set.  That is the verdict every workgroup reaches from
// the same totals anyway: the flag is set either by an earlier launch or by
// this launch's workgroup 0 from bit-identical sums.
__device__ __forceinline__ bool workgroup_stopped(int32_t seen) {
  __shared__ int32_t s_seen[kBlock / 64];
  if ((threadIdx.x & 63) == 0) s_seen[threadIdx.x >> 6] = seen;
  __syncthreads();
  int32_t any = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) any |= s_seen[w];
  return any != 0;
}

// Publish this workgroup's NV partial sums; returns true in every thread of
// the last workgroup to arrive, whose v[] (all threads) then holds the
// fixed-order total over all workgroups.
template <typename R, int NV>
__device__ __forceinline__ bool last_block_total(R (&v)[NV], R* __restrict__ partials, uint32_t* ticket) {
  __shared__ int s_last;
  __shared__ R s_tot[NV];
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) __hip_atomic_store(&partials[(size_t)blockIdx.x * NV + i], v[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const uint32_t prev = atomicAdd(ticket, 1u);
    s_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!s_last) return false;
  __threadfence();
  R acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = R(0);
  for (int b = threadIdx.x; b < (int)gridDim.x; b += kBlock)
#pragma unroll
    for (int i = 0; i < NV; ++i)
      acc[i] += __hip_atomic_load(&partials[(size_t)b * NV + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  block_sum<R, NV>(acc);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) s_tot[i] = acc[i];
    *ticket = 0u;  // ready for the next launch (kernel boundary orders it)
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = s_tot[i];
  return true;
}

// ----------------------------------------------------------------- COCG
// Scalar-block arithmetic is FP64 throughout; the complex64 recurrence
// accumulates its reductions in FP64 too (products of two floats are exact
// in double), since the unconjugated form r^T z cancels heavily.
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double s = fmax(fabs(b.x), fabs(b.y));
  const double br = b.x / s, bi = b.y / s;
  const double d = br * br + bi * bi;
  return make_double2((a.x * br + a.y * bi) / (d * s), (a.y * br - a.x * bi) / (d * s));
}
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// Per-workgroup partials of 4 sums -> partials[block][4] (plain stores; the
// consumer is a later kernel).
__device__ __forceinline__ void store_partials4(double (&v)[4], double* __restrict__ partials) {
  block_sum4(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) partials[(size_t)blockIdx.x * 4 + i] = v[i];
  }
}

// Every workgroup re-reduces the producer's nin partials in one fixed order,
// so all workgroups (and every run) see bit-identical totals.  Producers
// have at most 2048 workgroups: a thread's (up to) eight loads are issued
// together, then summed in order.
__device__ __forceinline__ void reduce_partials4(const double* __restrict__ partials, int nin, double (&t)[4]) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  double2 lo[8], hi[8];
  const double2* p2 = reinterpret_cast<const double2*>(partials);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int b = threadIdx.x + k * kBlock;
    lo[k] = b < nin ? p2[2 * (size_t)b] : make_double2(0.0, 0.0);
    hi[k] = b < nin ? p2[2 * (size_t)b + 1] : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (threadIdx.x + k * kBlock < nin) {
      acc[0] += lo[k].x;
      acc[1] += lo[k].y;
      acc[2] += hi[k].x;
      acc[3] += hi[k].y;
    }
  }
  for (int b = threadIdx.x + 8 * kBlock; b < nin; b += kBlock)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += partials[(size_t)b * 4 + i];
  block_sum4(acc);
#pragma unroll
  for (int i = 0; i < 4; ++i) t[i] = acc[i];
}

// Segment start: r = src (optionally x = 0), p = D^-1 r; rho = r^T p into
// slot par, rr, zz.  One writer (last workgroup).
template <typename R>
__global__ void __launch_bounds__(kBlock) k_cocg_init(int64_t n, const double2* __restrict__ src64,
                                                      const typename Cx<R>::T* __restrict__ dinv,
                                                      typename Cx<R>::T* __restrict__ x,
                                                      typename Cx<R>::T* __restrict__ r,
                                                      typename Cx<R>::T* __restrict__ p, CocgScalars* sc,
                                                      double* __restrict__ partials, int zero_x, int par) {
  using C = typename Cx<R>::T;
  if (sc->done) return;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const double2 s = src64[i];
    C ri = mk<C>(s.x, s.y);
    const C di = dinv[i];
    C zi;
    zi.x = di.x * ri.x - di.y * ri.y;
    zi.y = di.x * ri.y + di.y * ri.x;
    r[i] = ri;
    p[i] = zi;
    if (zero_x) x[i] = mk<C>(0.0, 0.0);
    v[0] += (double)ri.x * zi.x - (double)ri.y * zi.y;
    v[1] += (double)ri.x * zi.y + (double)ri.y * zi.x;
    v[2] += (double)ri.x * ri.x + (double)ri.y * ri.y;
    v[3] += (double)zi.x * zi.x + (double)zi.y * zi.y;
  }
  block_sum<double, 4>(v);
  if (!last_block_total<double, 4>(v, partials, &sc->ticket[0])) return;
  if (threadIdx.x == 0) {
    const double2 rho = make_double2(v[0], v[1]);
    const double rr = v[2], zz = v[3];
    sc->rho[par] = rho;
    sc->rr = rr;
    sc->rr_max[par] = rr;
    sc->iters[par] = sc->iters_out;
    if (sc->bb <= 0.0) sc->bb = rr;
    if (rr <= sc->tol2 * sc->bb) sc->done = 1;
    else if (cabs2(rho) <= sc->bd_tol * sc->bd_tol * rr * zz) sc->done = 3;
    if (sc->done) sc->stop_par = par;
  }
}

// q = A p; partials of p^T q (re, im), ||p||^2, ||q||^2.  No scalar writes.
template <typename R, typename VC = typename Cx<R>::T>
__global__ void __launch_bounds__(kBlock) k_cocg_spmv_dot(PatternDev pt, const VC* __restrict__ val,
                                                          const typename Cx<R>::T* __restrict__ p,
                                                          typename Cx<R>::T* __restrict__ q, const CocgScalars* sc,
                                                          double* __restrict__ partials) {
  using C = typename Cx<R>::T;
  // the stop flag is read here and tested together with the first row's
  // bounds, a scalar load the row has to wait for anyway, so launches queued
  // past convergence end before loading a row and working ones wait no longer.
  // No workgroup of this launch writes the flag (only the update kernels
  // do), so every wave reads the same value and a per-wave exit is safe.
  const int32_t stopped = sc->done;
  const int lane = threadIdx.x & 63;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  int nwaves;
  const int w = wave_row_start(nwaves);
  bool first = true;
  for (int32_t r0 = w; r0 < pt.nn; r0 += kRowsPerWave * nwaves) {
    int32_t rows[kRowsPerWave];
#pragma unroll
    for (int k = 0; k < kRowsPerWave; ++k) rows[k] = r0 + k * nwaves;
    R yr[kRowsPerWave], yi[kRowsPerWave];
    if (first) {
      const int32_t b0 = __builtin_amdgcn_readfirstlane(pt.row_ptr[rows[0]]);
      if (__builtin_amdgcn_readfirstlane(stopped) && b0 >= 0) return;
      first = false;
    }
    rows_product<R, kRowsPerWave, VC>(pt, val, p, rows, lane, yr, yi);
    if (lane == 0 || lane == 3 || lane == 6) {
#pragma unroll
      for (int k = 0; k < kRowsPerWave; ++k) {
        if (rows[k] >= pt.nn) continue;
        const size_t idx = 3 * (size_t)rows[k] + lane / 3;
        C o;
        o.x = yr[k];
        o.y = yi[k];
        q[idx] = o;
        const C pi = p[idx];
        v[0] += (double)pi.x * yr[k] - (double)pi.y * yi[k];
        v[1] += (double)pi.x * yi[k] + (double)pi.y * yr[k];
        v[2] += (double)pi.x * pi.x + (double)pi.y * pi.y;
        v[3] += (double)yr[k] * yr[k] + (double)yi[k] * yi[k];
      }
    }
  }
  if (__builtin_amdgcn_readfirstlane(stopped)) return;
  store_partials4(v, partials);
}

// alpha = rho / p^T q (re-reduced); x += alpha p; r -= alpha q;
// partials of rho' = r^T z (z = D^-1 r, not stored), ||r||^2, ||z||^2.
// A thread owns kPerThread entries kBlock apart per grid sweep; the first
// sweep's operands and the scalars are loaded before the re-reduction,
// which does not need them, so their latency overlaps it.
template <typename R>
__global__ void __launch_bounds__(kBlock) k_cocg_update(int64_t n, const typename Cx<R>::T* __restrict__ dinv,
                                                        typename Cx<R>::T* __restrict__ x,
                                                        typename Cx<R>::T* __restrict__ r,
                                                        const typename Cx<R>::T* __restrict__ p,
                                                        const typename Cx<R>::T* __restrict__ q, CocgScalars* sc,
                                                        const double* __restrict__ pin, int nin,
                                                        double* __restrict__ pout, int par) {
  using C = typename Cx<R>::T;
  const int32_t stopped = sc->done;
  const double2 rho = sc->rho[par];
  const double bd_tol = sc->bd_tol;
  const int64_t stride = (int64_t)gridDim.x * kBlock * kPerThread;
  int64_t i0 = (int64_t)blockIdx.x * kBlock * kPerThread + threadIdx.x;
  C pv[kPerThread], qv[kPerThread], dv[kPerThread], xv[kPerThread], rv[kPerThread];
  auto load = [&](int64_t b) {
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const int64_t i = b + (int64_t)k * kBlock;
      if (i < n) {
        pv[k] = p[i];
        qv[k] = q[i];
        dv[k] = dinv[i];
        xv[k] = x[i];
        rv[k] = r[i];
      }
    }
  };
  load(i0);
  // the stop flag is tested after the loads above are issued, as one
  // decision per workgroup (workgroup 0 of this launch may set it below)
  if (workgroup_stopped(__builtin_amdgcn_readfirstlane(stopped))) return;
  double t[4];
  reduce_partials4(pin, nin, t);
  const double2 pq = make_double2(t[0], t[1]);
  if (cabs2(pq) <= bd_tol * bd_tol * t[2] * t[3]) {
    // every workgroup reaches the same verdict; one records it
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->done = 3;
      sc->stop_par = par;
    }
    return;
  }
  const double2 alpha = cdiv(rho, pq);
  if (blockIdx.x == 0 && threadIdx.x == 0) sc->alpha = alpha;
  const R ar = (R)alpha.x, ai = (R)alpha.y;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  while (i0 < n) {
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const int64_t i = i0 + (int64_t)k * kBlock;
      if (i >= n) continue;
      const C pi = pv[k], qi = qv[k], di = dv[k];
      C xi = xv[k], ri = rv[k];
      xi.x += ar * pi.x - ai * pi.y;
      xi.y += ar * pi.y + ai * pi.x;
      ri.x -= ar * qi.x - ai * qi.y;
      ri.y -= ar * qi.y + ai * qi.x;
      x[i] = xi;
      r[i] = ri;
      const R zr = di.x * ri.x - di.y * ri.y;
      const R zi = di.x * ri.y + di.y * ri.x;
      v[0] += (double)ri.x * zr - (double)ri.y * zi;
      v[1] += (double)ri.x * zi + (double)ri.y * zr;
      v[2] += (double)ri.x * ri.x + (double)ri.y * ri.y;
      v[3] += (double)zr * zr + (double)zi * zi;
    }
    i0 += stride;
    if (i0 < n) load(i0);
  }
  store_partials4(v, pout);
}

// Re-reduce rho', ||r||^2, ||z||^2; decide (converged / iteration limit /
// breakdown / reliable update due) identically in every workgroup; if the
// recurrence continues, beta = rho' / rho and p = z + beta p.  Workgroup 0
// records the outcome; values read here live in slot par, values written
// for the next iteration in slot par ^ 1.
template <typename R>
__global__ void __launch_bounds__(kBlock) k_cocg_pupdate(int64_t n, const typename Cx<R>::T* __restrict__ dinv,
                                                         const typename Cx<R>::T* __restrict__ r,
                                                         typename Cx<R>::T* __restrict__ p, CocgScalars* sc,
                                                         const double* __restrict__ pin, int nin, int par) {
  using C = typename Cx<R>::T;
  const int32_t stopped = sc->done;
  // operands of the first sweep and the scalars first (as in the update)
  const int it = sc->iters[par] + 1;
  const double rmax = sc->rr_max[par];
  const double2 rho_old = sc->rho[par];
  const double tol2bb = sc->tol2 * sc->bb, bd_tol = sc->bd_tol, delta2 = sc->delta2;
  const int max_iters = sc->max_iters;
  const int64_t stride = (int64_t)gridDim.x * kBlock * kPerThread;
  int64_t i0 = (int64_t)blockIdx.x * kBlock * kPerThread + threadIdx.x;
  C dv[kPerThread], rv[kPerThread], pv[kPerThread];
  auto load = [&](int64_t b) {
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const int64_t i = b + (int64_t)k * kBlock;
      if (i < n) {
        dv[k] = dinv[i];
        rv[k] = r[i];
        pv[k] = p[i];
      }
    }
  };
  load(i0);
  if (workgroup_stopped(__builtin_amdgcn_readfirstlane(stopped))) return;
  double t[4];
  reduce_partials4(pin, nin, t);
  const double2 rho_new = make_double2(t[0], t[1]);
  const double rr = t[2], zz = t[3];
  int stop = 0;
  if (rr <= tol2bb) stop = 1;
  else if (it >= max_iters) stop = 2;
  else if (cabs2(rho_new) <= bd_tol * bd_tol * rr * zz) stop = 3;
  else if (delta2 > 0.0 && rr <= rmax && rr <= delta2 * rmax) stop = 4;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (stop) {
    // rho_{k-1} stays in slot par for the reliable update
    if (lead) {
      sc->iters[par ^ 1] = it;
      sc->iters_out = it;
      sc->rr = rr;
      sc->stop_par = par;
      sc->done = stop;
    }
    return;
  }
  const double2 beta = cdiv(rho_new, rho_old);
  if (lead) {
    sc->rho[par ^ 1] = rho_new;
    sc->rr_max[par ^ 1] = rr > rmax ? rr : rmax;
    sc->iters[par ^ 1] = it;
    sc->iters_out = it;
    sc->rr = rr;
    sc->beta = beta;
  }
  const R br = (R)beta.x, bi = (R)beta.y;
  while (i0 < n) {
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const int64_t i = i0 + (int64_t)k * kBlock;
      if (i >= n) continue;
      const C di = dv[k], ri = rv[k];
      C pi = pv[k];
      const R zr = di.x * ri.x - di.y * ri.y;
      const R zi = di.x * ri.y + di.y * ri.x;
      const R nr = zr + br * pi.x - bi * pi.y;
      const R ni = zi + br * pi.y + bi * pi.x;
      pi.x = nr;
      pi.y = ni;
      p[i] = pi;
    }
    i0 += stride;
    if (i0 < n) load(i0);
  }
}

// p = D^-1 r + beta p with beta from the scalar block (after a reliable
// update that kept the direction).
template <typename R>
__global__ void __launch_bounds__(kBlock) k_cocg_apply_beta(int64_t n, const typename Cx<R>::T* __restrict__ dinv,
                                                            const typename Cx<R>::T* __restrict__ r,
                                                            typename Cx<R>::T* __restrict__ p, const CocgScalars* sc) {
  using C = typename Cx<R>::T;
  if (sc->done) return;
  const R br = (R)sc->beta.x, bi = (R)sc->beta.y;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const C di = dinv[i], ri = r[i];
    C pi = p[i];
    const R zr = di.x * ri.x - di.y * ri.y;
    const R zi = di.x * ri.y + di.y * ri.x;
    const R nr = zr + br * pi.x - bi * pi.y;
    const R ni = zi + br * pi.y + bi * pi.x;
    pi.x = nr;
    pi.y = ni;
    p[i] = pi;
  }
}

// ---------------------------------------------- single-reduction COCG (FP64)
// The same Krylov iterates as COCG (section 3.1.5.1), reorganised so that one
// global reduction per iteration suffices: with z = D^-1 r and w = A z
// computed first, every scalar of the step follows from dot products of
// vectors available before the direction is updated:
//   gamma = r^T z,  delta = z^T w,  mu = z^T s_old          (s = A p)
//   beta  = -mu / pi_old   (makes p A-conjugate to p_old)
//   pi    = p^T s = delta + 2 beta mu + beta^2 pi_old       (A = A^T)
//   alpha = gamma / pi
//   p = z + beta p,  s = w + beta s,  x += alpha p,  z -= alpha D^-1 s.
// In exact arithmetic beta equals the COCG ratio of successive r^T z and pi
// the COCG denominator p^T A p.  Chronopoulos and Gear's single-reduction CG
// takes the conjugation from that recurrence instead (pi = delta - beta^2
// pi_old); on these indefinite systems it needs about 11 % more iterations
// than COCG, the explicit mu a few percent.  The product kernel
// (k_cocg_spmv_dot on z) yields delta; the update kernel yields gamma, mu,
// ||r||^2 and ||z||^2 of the next step, since it holds the new s and the new
// z of each entry.  One product and one update kernel make an iteration.
// The residual itself is not stored while iterating: the update carries z
// (the product's input) and forms r = D z entry by entry (D = 1 / D^-1) for
// r^T z and ||r||^2.

// Per-workgroup partials of 8 sums (gamma re/im, mu re/im, ||r||^2,
// ||z||^2, 0, 0) -> partials[block][8].
__device__ __forceinline__ void store_partials8(double (&v)[8], double* __restrict__ partials) {
  block_sum8(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) partials[(size_t)blockIdx.x * 8 + i] = v[i];
  }
}

// The sums a step needs, each in a fixed order: t[0..1] = z^T w from the
// product's na workgroups (the first two of its four values; its norms are
// not needed here), t[2..7] = gamma, mu, ||r||^2, ||z||^2 from the previous
// update's nb workgroups (eight values each, the last two unused).  All
// loads of a thread's first producers are issued before any is summed.
__device__ __forceinline__ void reduce_step_partials(const double* __restrict__ pa, int na,
                                                     const double* __restrict__ pb, int nb, double (&t)[8]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) t[i] = 0.0;
  const double2* a2 = reinterpret_cast<const double2*>(pa);
  const double2* b2 = reinterpret_cast<const double2*>(pb);
  double2 da[8], bq[3];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int b = threadIdx.x + k * kBlock;
    da[k] = b < na ? a2[2 * (size_t)b] : make_double2(0.0, 0.0);
  }
  const bool has_b = (int)threadIdx.x < nb;
#pragma unroll
  for (int k = 0; k < 3; ++k) bq[k] = has_b ? b2[4 * (size_t)threadIdx.x + k] : make_double2(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (threadIdx.x + k * kBlock < na) {
      t[0] += da[k].x;
      t[1] += da[k].y;
    }
  }
  for (int b = threadIdx.x + 8 * kBlock; b < na; b += kBlock) {
    t[0] += pa[(size_t)b * 4];
    t[1] += pa[(size_t)b * 4 + 1];
  }
  if (has_b)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      t[2 + 2 * k] += bq[k].x;
      t[3 + 2 * k] += bq[k].y;
    }
  for (int b = threadIdx.x + kBlock; b < nb; b += kBlock)
#pragma unroll
    for (int i = 0; i < 6; ++i) t[2 + i] += pb[(size_t)b * 8 + i];
  block_sum8(t);
}

// Segment start (r = the residual to restart from): z = D^-1 r, p = s = 0;
// the update kernel's partials of
// gamma, mu (= 0), ||r||^2, ||z||^2; pi_old = 0 in slot par marks the first
// step (beta = 0).  Same workgroup count as the update kernel.
__global__ void __launch_bounds__(kBlock) k_sr_init(int64_t n, const double2* __restrict__ r,
                                                    const double2* __restrict__ dinv, double2* __restrict__ z,
                                                    double2* __restrict__ p, double2* __restrict__ s,
                                                    CocgScalars* sc, double* __restrict__ pout, int par) {
  if (sc->done) return;
  double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const double2 ri = r[i], di = dinv[i];
    const double zr = di.x * ri.x - di.y * ri.y;
    const double zi = di.x * ri.y + di.y * ri.x;
    z[i] = make_double2(zr, zi);
    p[i] = make_double2(0.0, 0.0);
    s[i] = make_double2(0.0, 0.0);
    v[0] += ri.x * zr - ri.y * zi;
    v[1] += ri.x * zi + ri.y * zr;
    v[4] += ri.x * ri.x + ri.y * ri.y;
    v[5] += zr * zr + zi * zi;
  }
  store_partials8(v, pout);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->iters[par] = sc->iters_out;
    sc->rho[par] = make_double2(0.0, 0.0);
  }
}

// One step: reduce the product's partials (delta) and the previous step's
// (gamma, mu, ||r||^2, ||z||^2); decide convergence / iteration limit /
// breakdown identically in every workgroup; otherwise update p, s, x, z
// and emit the next step's partials.  Slot par holds pi_old and the
// iteration count; slot par ^ 1 receives pi and the count.  Breakdown:
// gamma negligible against ||r|| ||z||, or pi lost to cancellation among its
// three terms (or zero / not finite).
__global__ void __launch_bounds__(kBlock) k_sr_update(int64_t n, const double2* __restrict__ dinv,
                                                      double2* __restrict__ x,
                                                      double2* __restrict__ z, const double2* __restrict__ w,
                                                      double2* __restrict__ p, double2* __restrict__ s,
                                                      CocgScalars* sc, const double* __restrict__ pin_a, int nin_a,
                                                      const double* __restrict__ pin_b, int nin_b,
                                                      double* __restrict__ pout, int par) {
  const int32_t stopped = sc->done;
  const double2 pi_old = sc->rho[par];
  const int it = sc->iters[par];
  const double tol2bb = sc->tol2 * sc->bb, bd_tol = sc->bd_tol;
  const int max_iters = sc->max_iters;
  const int64_t stride = (int64_t)gridDim.x * kBlock * kPerThread;
  int64_t i0 = (int64_t)blockIdx.x * kBlock * kPerThread + threadIdx.x;
  double2 zv[kPerThread], wv[kPerThread], pv[kPerThread], sv[kPerThread], xv[kPerThread], dv[kPerThread];
  auto load = [&](int64_t b) {
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const int64_t i = b + (int64_t)k * kBlock;
      if (i < n) {
        zv[k] = z[i];
        wv[k] = w[i];
        pv[k] = p[i];
        sv[k] = s[i];
        xv[k] = x[i];
        dv[k] = dinv[i];
      }
    }
  };
  load(i0);
  if (workgroup_stopped(__builtin_amdgcn_readfirstlane(stopped))) return;
  double t[8];
  reduce_step_partials(pin_a, nin_a, pin_b, nin_b, t);
  const double2 delta = make_double2(t[0], t[1]);
  const double2 gamma = make_double2(t[2], t[3]), mu = make_double2(t[4], t[5]);
  const double rr = t[6], zz = t[7];
  int stop = 0;
  double2 beta = make_double2(0.0, 0.0), pi = delta;
  if (rr <= tol2bb) stop = 1;
  else if (it >= max_iters) stop = 2;
  else if (cabs2(gamma) <= bd_tol * bd_tol * rr * zz) stop = 3;
  if (!stop) {
    double mag = sqrt(cabs2(delta));
    if (pi_old.x != 0.0 || pi_old.y != 0.0) {
      const double2 b = cdiv(mu, pi_old);
      beta = make_double2(-b.x, -b.y);
      const double2 bm = make_double2(beta.x * mu.x - beta.y * mu.y, beta.x * mu.y + beta.y * mu.x);
      const double2 b2 = make_double2(beta.x * beta.x - beta.y * beta.y, 2.0 * beta.x * beta.y);
      const double2 bbp = make_double2(b2.x * pi_old.x - b2.y * pi_old.y, b2.x * pi_old.y + b2.y * pi_old.x);
      pi = make_double2(delta.x + 2.0 * bm.x + bbp.x, delta.y + 2.0 * bm.y + bbp.y);
      mag += 2.0 * sqrt(cabs2(bm)) + sqrt(cabs2(bbp));
    }
    if (!(sqrt(cabs2(pi)) > bd_tol * mag)) stop = 3;
  }
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (stop) {
    if (lead) {
      sc->iters[par ^ 1] = it;
      sc->iters_out = it;
      sc->rr = rr;
      sc->stop_par = par;
      sc->done = stop;
    }
    return;
  }
  const double2 alpha = cdiv(gamma, pi);
  if (lead) {
    sc->rho[par ^ 1] = pi;
    sc->iters[par ^ 1] = it + 1;
    sc->iters_out = it + 1;
    sc->rr = rr;
    sc->alpha = alpha;
    sc->beta = beta;
  }
  const double ar = alpha.x, ai = alpha.y, br = beta.x, bi = beta.y;
  double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  while (i0 < n) {
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const int64_t i = i0 + (int64_t)k * kBlock;
      if (i >= n) continue;
      const double2 zi = zv[k], wi = wv[k], po = pv[k], so = sv[k], di = dv[k];
      const double2 pn = make_double2(zi.x + br * po.x - bi * po.y, zi.y + br * po.y + bi * po.x);
      const double2 sn = make_double2(wi.x + br * so.x - bi * so.y, wi.y + br * so.y + bi * so.x);
      double2 xi = xv[k];
      xi.x += ar * pn.x - ai * pn.y;
      xi.y += ar * pn.y + ai * pn.x;
      // z -= alpha D^-1 s
      const double2 as = make_double2(ar * sn.x - ai * sn.y, ar * sn.y + ai * sn.x);
      const double zr = zi.x - (di.x * as.x - di.y * as.y);
      const double zim = zi.y - (di.x * as.y + di.y * as.x);
      // r = D z with D = 1 / D^-1
      const double inv = 1.0 / (di.x * di.x + di.y * di.y);
      const double2 ri = make_double2((di.x * zr + di.y * zim) * inv, (di.x * zim - di.y * zr) * inv);
      p[i] = pn;
      s[i] = sn;
      x[i] = xi;
      z[i] = make_double2(zr, zim);
      v[0] += ri.x * zr - ri.y * zim;
      v[1] += ri.x * zim + ri.y * zr;
      v[2] += zr * sn.x - zim * sn.y;
      v[3] += zr * sn.y + zim * sn.x;
      v[4] += ri.x * ri.x + ri.y * ri.y;
      v[5] += zr * zr + zim * zim;
    }
    i0 += stride;
    if (i0 < n) load(i0);
  }
  store_partials8(v, pout);
}

// Reliable update (complex64 recurrence), see the launcher's comment.
__global__ void __launch_bounds__(kBlock) k_cocg_rescale(int64_t n, const double2* __restrict__ r64, double inv_s,
                                                         const float2* __restrict__ dinv, float2* __restrict__ r,
                                                         float2* __restrict__ p, CocgScalars* sc,
                                                         double* __restrict__ partials, double ratio, double tol2,
                                                         int fresh, int par) {
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const double2 s = r64[i];
    const float2 ri = make_float2((float)(s.x * inv_s), (float)(s.y * inv_s));
    const float2 di = dinv[i];
    const float zr = di.x * ri.x - di.y * ri.y;
    const float zi = di.x * ri.y + di.y * ri.x;
    r[i] = ri;
    if (fresh) p[i] = make_float2(zr, zi);
    v[0] += (double)ri.x * zr - (double)ri.y * zi;
    v[1] += (double)ri.x * zi + (double)ri.y * zr;
    v[2] += (double)ri.x * ri.x + (double)ri.y * ri.y;
    v[3] += (double)zr * zr + (double)zi * zi;
  }
  block_sum<double, 4>(v);
  if (!last_block_total<double, 4>(v, partials, &sc->ticket[3])) return;
  if (threadIdx.x == 0) {
    const double2 rho_new = make_double2(v[0], v[1]);
    const double rr = v[2], zz = v[3];
    sc->tol2 = tol2;
    sc->rr = rr;
    sc->rr_max[par] = rr;
    sc->iters[par] = sc->iters_out;
    sc->done = 0;
    if (cabs2(rho_new) <= sc->bd_tol * sc->bd_tol * rr * zz) {
      sc->done = 3;
      sc->stop_par = par;
    } else if (!fresh) {
      const double2 old = sc->rho[sc->stop_par];
      sc->beta = cdiv(rho_new, make_double2(old.x * ratio, old.y * ratio));
    }
    sc->rho[par] = rho_new;
  }
}

// Reliable update of an FP64 recurrence whose residual buffer has just been
// overwritten with the true residual: rho' = r^T D^-1 r, beta = rho' /
// rho_{k-1} (the caller then applies beta to the direction).
__global__ void __launch_bounds__(kBlock) k_cocg_replace(int64_t n, const double2* __restrict__ r,
                                                         const double2* __restrict__ dinv, CocgScalars* sc,
                                                         double* __restrict__ partials, int par) {
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const double2 ri = r[i], di = dinv[i];
    const double zr = di.x * ri.x - di.y * ri.y;
    const double zi = di.x * ri.y + di.y * ri.x;
    v[0] += ri.x * zr - ri.y * zi;
    v[1] += ri.x * zi + ri.y * zr;
    v[2] += ri.x * ri.x + ri.y * ri.y;
    v[3] += zr * zr + zi * zi;
  }
  block_sum<double, 4>(v);
  if (!last_block_total<double, 4>(v, partials, &sc->ticket[3])) return;
  if (threadIdx.x == 0) {
    const double2 rho_new = make_double2(v[0], v[1]);
    sc->rr = v[2];
    sc->rr_max[par] = v[2];
    sc->iters[par] = sc->iters_out;
    sc->done = 0;
    if (cabs2(rho_new) <= sc->bd_tol * sc->bd_tol * v[2] * v[3]) {
      sc->done = 3;
      sc->stop_par = par;
    } else {
      sc->beta = cdiv(rho_new, sc->rho[sc->stop_par]);
    }
    sc->rho[par] = rho_new;
  }
}

__global__ void __launch_bounds__(kBlock) k_ir_fold(int64_t n, float2* __restrict__ d, double s,
                                                    double2* __restrict__ x) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const float2 di = d[i];
    double2 xi = x[i];
    xi.x += s * (double)di.x;
    xi.y += s * (double)di.y;
    x[i] = xi;
    d[i] = make_float2(0.f, 0.f);
  }
}

// r = b - A x (FP64) with ||r||^2
__global__ void __launch_bounds__(kBlock) k_residual(PatternDev pt, const double2* __restrict__ val,
                                                     const double2* __restrict__ x, const double2* __restrict__ b,
                                                     double2* __restrict__ r, double* __restrict__ partials,
                                                     uint32_t* ticket, double* rr_out) {
  const int lane = threadIdx.x & 63;
  double v[1] = {0.0};
  int nwaves;
  const int w = wave_row_start(nwaves);
  for (int32_t r0 = w; r0 < pt.nn; r0 += kRowsPerWave * nwaves) {
    int32_t rows[kRowsPerWave];
#pragma unroll
    for (int k = 0; k < kRowsPerWave; ++k) rows[k] = r0 + k * nwaves;
    double yr[kRowsPerWave], yi[kRowsPerWave];
    rows_product<double, kRowsPerWave>(pt, val, x, rows, lane, yr, yi);
    if (lane == 0 || lane == 3 || lane == 6) {
#pragma unroll
      for (int k = 0; k < kRowsPerWave; ++k) {
        if (rows[k] >= pt.nn) continue;
        const size_t idx = 3 * (size_t)rows[k] + lane / 3;
        const double2 bi = b[idx];
        const double2 ri = make_double2(bi.x - yr[k], bi.y - yi[k]);
        r[idx] = ri;
        v[0] += ri.x * ri.x + ri.y * ri.y;
      }
    }
  }
  block_sum<double, 1>(v);
  if (!last_block_total<double, 1>(v, partials, ticket)) return;
  if (threadIdx.x == 0) *rr_out = v[0];
}

__global__ void __launch_bounds__(kBlock) k_norm2(int64_t n, const double2* __restrict__ a, double* __restrict__ partials,
                                                  uint32_t* ticket, double* out) {
  double v[1] = {0.0};
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const double2 t = a[i];
    v[0] += t.x * t.x + t.y * t.y;
  }
  block_sum<double, 1>(v);
  if (!last_block_total<double, 1>(v, partials, ticket)) return;
  if (threadIdx.x == 0) *out = v[0];
}

}  // namespace

namespace k {

int reduce_blocks_for(int64_t n) {
  int64_t b = (n + kBlock * kPerThread - 1) / (kBlock * kPerThread);
  if (b < 8) b = 8;
  if (b > 2048) b = 2048;
  return (int)((b + 7) / 8 * 8);
}

SpmvLaunch spmv_launch_for(int32_t nn, int n_cu) {
  // enough waves to cover the rows once, capped at 8 workgroups per CU
  int64_t b = ((int64_t)nn + kWavesPerBlock * kRowsPerWave - 1) / (kWavesPerBlock * kRowsPerWave);
  int64_t cap = (int64_t)n_cu * 8;
  if (cap > 2048) cap = 2048;  // partial-sum buffers hold 2048 workgroups
  if (b > cap) b = cap;
  if (b < 8) b = 8;
  SpmvLaunch L;
  L.blocks = (int)((b + 7) / 8 * 8);
  return L;
}

hipError_t spmv_half_c128(hipStream_t st, const PatternDev& p, const double2* hval, const int32_t* hpos,
                          const double2* x, double2* y, SpmvLaunch L) {
  hipLaunchKernelGGL((k_spmv_half<double>), dim3(L.blocks), dim3(kBlock), 0, st, p, hval, hpos, x, y);
  return hipGetLastError();
}

hipError_t gather_half(hipStream_t st, int64_t nnzb, const int32_t* hpos, const double2* val, double2* hval) {
  const int64_t t = nnzb * 9;
  hipLaunchKernelGGL(k_gather_half, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, nnzb, hpos, val, hval);
  return hipGetLastError();
}

hipError_t spmv_c128(hipStream_t st, const PatternDev& p, const double2* val, const double2* x, double2* y,
                     SpmvLaunch L) {
  if (p.nn == 0) return hipSuccess;
  hipLaunchKernelGGL(k_spmv<double>, dim3(L.blocks), dim3(kBlock), 0, st, p, val, x, y);
  return hipGetLastError();
}

hipError_t spmv_m32(hipStream_t st, const PatternDev& p, const float2* val, const double2* x, double2* y,
                    SpmvLaunch L) {
  if (p.nn == 0) return hipSuccess;
  hipLaunchKernelGGL((k_spmv<double, float2>), dim3(L.blocks), dim3(kBlock), 0, st, p, val, x, y);
  return hipGetLastError();
}

hipError_t cocg_spmv_dot_m32(hipStream_t st, const PatternDev& pt, const float2* val, const double2* p, double2* q,
                             CocgScalars* sc, void* partials, SpmvLaunch L) {
  hipLaunchKernelGGL((k_cocg_spmv_dot<double, float2>), dim3(L.blocks), dim3(kBlock), 0, st, pt, val, p, q, sc,
                     reinterpret_cast<double*>(partials));
  return hipGetLastError();
}

hipError_t cocg_replace_c128(hipStream_t st, int64_t n, const double2* r, const double2* dinv, CocgScalars* sc,
                             void* partials, int par) {
  hipLaunchKernelGGL(k_cocg_replace, dim3(reduce_blocks_for(n)), dim3(kBlock), 0, st, n, r, dinv, sc,
                     reinterpret_cast<double*>(partials), par);
  return hipGetLastError();
}

hipError_t spmv_c64(hipStream_t st, const PatternDev& p, const float2* val, const float2* x, float2* y,
                    SpmvLaunch L) {
  if (p.nn == 0) return hipSuccess;
  hipLaunchKernelGGL(k_spmv<float>, dim3(L.blocks), dim3(kBlock), 0, st, p, val, x, y);
  return hipGetLastError();
}

int update_blocks_for(int64_t n) { return reduce_blocks_for(n); }

hipError_t cocg_init_c128(hipStream_t st, int64_t n, const double2* b, const double2* dinv, double2* x, double2* r,
                          double2* p, CocgScalars* sc, void* partials, int zero_x, int par) {
  hipLaunchKernelGGL(k_cocg_init<double>, dim3(reduce_blocks_for(n)), dim3(kBlock), 0, st, n, b, dinv, x, r, p, sc,
                     reinterpret_cast<double*>(partials), zero_x, par);
  return hipGetLastError();
}

hipError_t cocg_spmv_dot_c128(hipStream_t st, const PatternDev& pt, const double2* val, const double2* p, double2* q,
                              CocgScalars* sc, void* partials, SpmvLaunch L) {
  hipLaunchKernelGGL((k_cocg_spmv_dot<double>), dim3(L.blocks), dim3(kBlock), 0, st, pt, val, p, q, sc,
                     reinterpret_cast<double*>(partials));
  return hipGetLastError();
}

hipError_t sr_init_c128(hipStream_t st, int64_t n, const double2* r, const double2* dinv, double2* z, double2* p,
                        double2* s, CocgScalars* sc, void* partials_out, int par) {
  hipLaunchKernelGGL(k_sr_init, dim3(reduce_blocks_for(n)), dim3(kBlock), 0, st, n, r, dinv, z, p, s, sc,
                     reinterpret_cast<double*>(partials_out), par);
  return hipGetLastError();
}

hipError_t sr_update_c128(hipStream_t st, int64_t n, const double2* dinv, double2* x, double2* z, const double2* w,
                          double2* p, double2* s, CocgScalars* sc, const void* partials_a, int nin_a,
                          const void* partials_b, void* partials_out, int par) {
  const int nb = reduce_blocks_for(n);
  hipLaunchKernelGGL(k_sr_update, dim3(nb), dim3(kBlock), 0, st, n, dinv, x, z, w, p, s, sc,
                     reinterpret_cast<const double*>(partials_a), nin_a,
                     reinterpret_cast<const double*>(partials_b), nb, reinterpret_cast<double*>(partials_out), par);
  return hipGetLastError();
}

hipError_t cocg_update_c128(hipStream_t st, int64_t n, const double2* dinv, double2* x, double2* r, const double2* p,
                            const double2* q, CocgScalars* sc, const void* pin, int nin, void* pout, int par) {
  hipLaunchKernelGGL(k_cocg_update<double>, dim3(reduce_blocks_for(n)), dim3(kBlock), 0, st, n, dinv, x, r, p, q, sc,
                     reinterpret_cast<const double*>(pin), nin, reinterpret_cast<double*>(pout), par);
  return hipGetLastError();
}

hipError_t cocg_pupdate_c128(hipStream_t st, int64_t n, const double2* dinv, const double2* r, double2* p,
                             CocgScalars* sc, const void* pin, int par) {
  hipLaunchKernelGGL(k_cocg_pupdate<double>, dim3(reduce_blocks_for(n)), dim3(kBlock), 0, st, n, dinv, r, p, sc,
                     reinterpret_cast<const double*>(pin), reduce_blocks_for(n), par);
  return hipGetLastError();
}

hipError_t cocg_apply_beta_c128(hipStream_t st, int64_t n, const double2* dinv, const double2* r, double2* p,
                                const CocgScalars* sc) {
  hipLaunchKernelGGL(k_cocg_apply_beta<double>, dim3(reduce_blocks_for(n)), dim3(kBlock), 0, st, n, dinv, r, p, sc);
  return hipGetLastError();
}

hipError_t cocg_spmv_dot_c64(hipStream_t st, const PatternDev& pt, const float2* val, const float2* p, float2* q,
                             CocgScalars* sc, void* partials, SpmvLaunch L) {
  hipLaunchKernelGGL((k_cocg_spmv_dot<float>), dim3(L.blocks), dim3(kBlock), 0, st, pt, val, p, q, sc,
                     reinterpret_cast<double*>(partials));
  return hipGetLastError();
}

hipError_t cocg_update_c64(hipStream_t st, int64_t n, const float2* dinv, float2* x, float2* r, const float2* p,
                           const float2* q, CocgScalars* sc, const void* pin, int nin, void* pout, int par) {
  hipLaunchKernelGGL(k_cocg_update<float>, dim3(reduce_blocks_for(n)), dim3(kBlock), 0, st, n, dinv, x, r, p, q, sc,
                     reinterpret_cast<const double*>(pin), nin, reinterpret_cast<double*>(pout), par);
  return hipGetLastError();
}

hipError_t cocg_pupdate_c64(hipStream_t st, int64_t n, const float2* dinv, const float2* r, float2* p,
                            CocgScalars* sc, const void* pin, int par) {
  hipLaunchKernelGGL(k_cocg_pupdate<float>, dim3(reduce_blocks_for(n)), dim3(kBlock), 0, st, n, dinv, r, p, sc,
                     reinterpret_cast<const double*>(pin), reduce_blocks_for(n), par);
  return hipGetLastError();
}

hipError_t cocg_apply_beta_c64(hipStream_t st, int64_t n, const float2* dinv, const float2* r, float2* p,
                               const CocgScalars* sc) {
  hipLaunchKernelGGL(k_cocg_apply_beta<float>, dim3(reduce_blocks_for(n)), dim3(kBlock), 0, st, n, dinv, r, p, sc);
  return hipGetLastError();
}

hipError_t cocg_rescale_c64(hipStream_t st, int64_t n, const double2* r64, double inv_s, const float2* dinv, float2* r,
                            float2* p, CocgScalars* sc, void* partials, double ratio, double tol2, int fresh, int par) {
  hipLaunchKernelGGL(k_cocg_rescale, dim3(reduce_blocks_for(n)), dim3(kBlock), 0, st, n, r64, inv_s, dinv, r, p, sc,
                     reinterpret_cast<double*>(partials), ratio, tol2, fresh, par);
  return hipGetLastError();
}

hipError_t ir_fold(hipStream_t st, int64_t n, float2* d, double s, double2* x) {
  hipLaunchKernelGGL(k_ir_fold, dim3(reduce_blocks_for(n)), dim3(kBlock), 0, st, n, d, s, x);
  return hipGetLastError();
}

hipError_t residual_c128(hipStream_t st, const PatternDev& pt, const double2* val, const double2* x, const double2* b,
                         double2* r, double* partials, uint32_t* ticket, double* rr_out, SpmvLaunch L) {
  hipLaunchKernelGGL(k_residual, dim3(L.blocks), dim3(kBlock), 0, st, pt, val, x, b, r, partials, ticket, rr_out);
  return hipGetLastError();
}

hipError_t norm2_c128(hipStream_t st, int64_t n, const double2* v, double* partials, uint32_t* ticket, double* out) {
  hipLaunchKernelGGL(k_norm2, dim3(reduce_blocks_for(n)), dim3(kBlock), 0, st, n, v, partials, ticket, out);
  return hipGetLastError();
}

}  // namespace k
}  // namespace femh
