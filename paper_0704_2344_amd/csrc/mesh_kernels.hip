// Device kernels for the structured hexahedral mesh: active-node numbering,
// the 3x3-block sparsity pattern, owner-computes assembly of eqs. (1)-(4),
// right-hand sides of eq. (4), the output scatter, and a copy probe.
//
// Assembly follows the paper's "assembly by degree of freedom" (section
// 3.1.2): each block (a, b) is produced by one thread from the (at most 8)
// elements containing both nodes, so no two threads write the same entry and
// no symbolic phase or atomics are needed.  On the uniform box every element
// matrix is a combination of closed-form Kronecker products of 1-D
// integrals, which the thread evaluates on the fly.
#include "internal.h"

namespace femh {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cinv(double2 a) {
  // 1 / a with scaling against overflow
  double s = fabs(a.x) > fabs(a.y) ? fabs(a.x) : fabs(a.y);
  double ar = a.x / s, ai = a.y / s;
  double d = ar * ar + ai * ai;
  return make_double2(ar / (d * s), -ai / (d * s));
}

// ----------------------------------------------------------------- scan
__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const int32_t* __restrict__ in,
                                                              int32_t* __restrict__ out, int64_t n,
                                                              int32_t* __restrict__ tile_sums) {
  __shared__ int32_t s_warp[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int32_t v[kScanItems];
  int32_t local = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + i;
    v[i] = idx < n ? in[idx] : 0;
    local += v[i];
  }
  // inclusive scan of `local` over the block: wave scan then wave offsets
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int32_t incl = local;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int32_t t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  if (lane == 63) s_warp[wid] = incl;
  __syncthreads();
  int32_t wave_off = 0;
  for (int w = 0; w < wid; ++w) wave_off += s_warp[w];
  int32_t run = wave_off + incl - local;  // exclusive prefix of this thread
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + i;
    if (idx < n) out[idx] = run;
    run += v[i];
  }
  if (threadIdx.x == kScanThreads - 1) tile_sums[blockIdx.x] = wave_off + incl;
}

__global__ void k_scan_add(int32_t* __restrict__ out, int64_t n, const int32_t* __restrict__ tile_off) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  const int32_t add = tile_off[blockIdx.x];
  for (int i = threadIdx.x; i < kScanTile; i += blockDim.x) {
    int64_t idx = base + i;
    if (idx < n) out[idx] += add;
  }
}

__global__ void k_scan_total(const int32_t* in, const int32_t* out, int64_t n, int32_t* total) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *total = n > 0 ? out[n - 1] + in[n - 1] : 0;
}

// ------------------------------------------------------------ materials
__global__ void k_check_materials(const double2* __restrict__ eps, const double2* __restrict__ mu,
                                  int64_t ne, int32_t* flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ne) return;
  int bad = 0;
  if (eps) {
    double2 e = eps[i];
    if (!isfinite(e.x) || !isfinite(e.y)) bad |= 1;
    else if (e.x == 0.0 && e.y == 0.0) bad |= 2;
  }
  if (mu) {
    double2 m = mu[i];
    if (!isfinite(m.x) || !isfinite(m.y)) bad |= 1;
  }
  if (bad) atomicOr(flag, bad);
}

// ------------------------------------------------------------- numbering
__device__ __forceinline__ bool elem_active(const MeshDev& m, int ex, int ey, int ez) {
  if (ex < 0 || ey < 0 || ez < 0 || ex >= m.nx || ey >= m.ny || ez >= m.nz) return false;
  if (!m.pec) return true;
  return m.pec[(int64_t)ex + (int64_t)m.nx * (ey + (int64_t)m.ny * ez)] == 0;
}

__global__ void k_node_flags(MeshDev m, int32_t* __restrict__ flags) {
  const int64_t gx = m.nx + 1, gy = m.ny + 1, gz = m.nz + 1;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= gx * gy * gz) return;
  const int i = (int)(g % gx), j = (int)((g / gx) % gy), kk = (int)(g / (gx * gy));
  int act = 0;
  for (int dz = -1; dz <= 0 && !act; ++dz)
    for (int dy = -1; dy <= 0 && !act; ++dy)
      for (int dx = -1; dx <= 0 && !act; ++dx) act = elem_active(m, i + dx, j + dy, kk + dz);
  flags[g] = act;
}

__global__ void k_node_compact(int64_t ngrid, const int32_t* __restrict__ flags,
                               const int32_t* __restrict__ scan, int32_t* __restrict__ node_id,
                               int32_t* __restrict__ node_grid) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngrid) return;
  if (flags[g]) {
    const int32_t id = scan[g];
    node_id[g] = id;
    node_grid[id] = (int32_t)g;
  } else {
    node_id[g] = -1;
  }
}

// Does the element box shared by node (i,j,k) and its neighbour at offset
// (dx,dy,dz) contain an active element?  Along an axis with offset 0 the
// two nodes share elements on both sides; with offset +-1 only the one
// element between them.
__device__ __forceinline__ bool share_active(const MeshDev& m, int i, int j, int kk, int dx, int dy,
                                             int dz) {
  const int x0 = dx == 0 ? i - 1 : (dx > 0 ? i : i - 1), x1 = dx == 0 ? i : x0;
  const int y0 = dy == 0 ? j - 1 : (dy > 0 ? j : j - 1), y1 = dy == 0 ? j : y0;
  const int z0 = dz == 0 ? kk - 1 : (dz > 0 ? kk : kk - 1), z1 = dz == 0 ? kk : z0;
  for (int ez = z0; ez <= z1; ++ez)
    for (int ey = y0; ey <= y1; ++ey)
      for (int ex = x0; ex <= x1; ++ex)
        if (elem_active(m, ex, ey, ez)) return true;
  return false;
}

__global__ void k_row_masks(MeshDev m, int32_t nn, const int32_t* __restrict__ node_grid,
                            uint32_t* __restrict__ mask, int32_t* __restrict__ counts) {
  const int32_t a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nn) return;
  const int64_t gx = m.nx + 1, gy = m.ny + 1;
  const int64_t g = node_grid[a];
  const int i = (int)(g % gx), j = (int)((g / gx) % gy), kk = (int)(g / (gx * gy));
  uint32_t bits = 0;
  for (int slot = 0; slot < 27; ++slot) {
    const int dx = slot % 3 - 1, dy = (slot / 3) % 3 - 1, dz = slot / 9 - 1;
    if (share_active(m, i, j, kk, dx, dy, dz)) bits |= 1u << slot;
  }
  mask[a] = bits;
  counts[a] = __popc(bits);
}

// ------------------------------------------------------------- assembly
// 1-D integrals on [0, h] of the linear functions N_0 = 1 - t/h, N_1 = t/h:
//   mass   int N_a N_b     = h/6 (2 if a == b else 1)
//   stiff  int N_a' N_b'   = (1 if a == b else -1) / h
//   mixed  int N_a' N_b    = -1/2 (a = 0), +1/2 (a = 1)
__device__ __forceinline__ double m1(int a, int b, double h) { return h * (a == b ? (1.0 / 3.0) : (1.0 / 6.0)); }
__device__ __forceinline__ double k1(int a, int b, double h) { return (a == b ? 1.0 : -1.0) / h; }
__device__ __forceinline__ double g1(int a) { return a ? 0.5 : -0.5; }

// Components of the node at grid index gi fixed to zero by the plane faces
// (section 3.1.3): bit c set = component c.  A symmetry face fixes the
// component along its normal (n . H = 0), an antisymmetry face the two
// tangential ones (n x H = 0).
__device__ __forceinline__ int fixed_components(const MeshDev& m, const int (&gi)[3]) {
  const int planes = m.sym_mask | m.anti_mask;
  if (!planes) return 0;
  const int nel[3] = {m.nx, m.ny, m.nz};
  int cm = 0;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    if (!((planes >> f) & 1)) continue;
    const int ax = f >> 1, side = f & 1;
    if (gi[ax] != (side ? nel[ax] : 0)) continue;
    cm |= ((m.sym_mask >> f) & 1) ? (1 << ax) : (7 & ~(1 << ax));
  }
  return cm;
}

__global__ void __launch_bounds__(256) k_assemble(MeshDev m, PatternDev p, int32_t* __restrict__ col_idx,
                                                  double2* __restrict__ val64, float2* __restrict__ val32,
                                                  double2* __restrict__ dinv64, float2* __restrict__ dinv32) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t a = (int32_t)(t >> 5);
  const int slot = (int)(t & 31);
  if (a >= p.nn || slot >= 27) return;
  const uint32_t bits = p.nbr_mask[a];
  if (!((bits >> slot) & 1u)) return;
  const int64_t pos = (int64_t)p.row_ptr[a] + __popc(bits & ((1u << slot) - 1u));
  const int d[3] = {slot % 3 - 1, (slot / 3) % 3 - 1, slot / 9 - 1};
  const int64_t gx = m.nx + 1, gy = m.ny + 1;
  const int64_t g = p.node_grid[a];
  const int gi[3] = {(int)(g % gx), (int)((g / gx) % gy), (int)(g / (gx * gy))};
  const int nel[3] = {m.nx, m.ny, m.nz};
  const int64_t gb = g + d[0] + gx * (d[1] + gy * (int64_t)d[2]);
  col_idx[pos] = p.node_id[gb];

  double2 K[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) K[i][j] = make_double2(0.0, 0.0);

  int lo[3], hi[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    lo[ax] = d[ax] == 0 ? gi[ax] - 1 : (d[ax] > 0 ? gi[ax] : gi[ax] - 1);
    hi[ax] = d[ax] == 0 ? gi[ax] : lo[ax];
    if (lo[ax] < 0) lo[ax] = 0;
    if (hi[ax] > nel[ax] - 1) hi[ax] = nel[ax] - 1;
  }
  for (int ez = lo[2]; ez <= hi[2]; ++ez)
    for (int ey = lo[1]; ey <= hi[1]; ++ey)
      for (int ex = lo[0]; ex <= hi[0]; ++ex) {
        const int64_t e = ex + (int64_t)m.nx * (ey + (int64_t)m.ny * ez);
        if (m.pec && m.pec[e]) continue;
        const int ee[3] = {ex, ey, ez};
        int la[3], lb[3];
        double mm[3], kk[3], ga[3], gbv[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          la[ax] = gi[ax] - ee[ax];
          lb[ax] = la[ax] + d[ax];
          mm[ax] = m1(la[ax], lb[ax], m.h[ax]);
          kk[ax] = k1(la[ax], lb[ax], m.h[ax]);
          ga[ax] = g1(la[ax]);
          gbv[ax] = g1(lb[ax]);
        }
        // G[p][q] = int dN_a/dx_p dN_b/dx_q : product over axes of the 1-D
        // factor (stiff on p == q == axis, mixed on the derivative axis of
        // a or of b, mass elsewhere).
        double G[3][3];
#pragma unroll
        for (int pp = 0; pp < 3; ++pp)
#pragma unroll
          for (int qq = 0; qq < 3; ++qq) {
            double v = 1.0;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
              double f;
              if (ax == pp && ax == qq) f = kk[ax];
              else if (ax == pp) f = ga[ax];
              else if (ax == qq) f = gbv[ax];
              else f = mm[ax];
              v *= f;
            }
            G[pp][qq] = v;
          }
        const double M = mm[0] * mm[1] * mm[2];
        const double trG = G[0][0] + G[1][1] + G[2][2];
        const double2 ie = m.eps ? cinv(m.eps[e]) : make_double2(1.0, 0.0);
        const double2 mu = m.mu ? m.mu[e] : make_double2(1.0, 0.0);
        const double2 mass = cscale(mu, -m.k0 * m.k0 * M);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            // (1/eps) (delta_ij trG - G_ji) + s G_ij - k0^2 mu delta_ij M
            const double curl = (i == j ? trG : 0.0) - G[j][i];
            double2 v = cadd(cscale(ie, curl), make_double2(m.s * G[i][j], 0.0));
            if (i == j) v = cadd(v, mass);
            K[i][j] = cadd(K[i][j], v);
          }
        // The printed penalty surface term (paper-literal variant), averaged
        // with its transpose: on each face of the element that lies on an
        // ABC outer face or against a PEC element, with outward normal along
        // axis ax (sign sg), the term's row (a, ax) holds
        // -s sg int N_a dN_b/dx_j dS in column (b, j); its transpose adds
        // -s sg int N_b dN_a/dx_i dS at (a, i), (b, ax).  Half of each.
        if (m.penalty_surface) {
#pragma unroll
          for (int f = 0; f < 6; ++f) {
            const int ax = f >> 1, side = f & 1;
            const int nbr = ee[ax] + (side ? 1 : -1);
            bool on;
            if (nbr < 0 || nbr >= nel[ax]) {
              on = (m.abc_mask >> f) & 1;
            } else {
              int en[3] = {ee[0], ee[1], ee[2]};
              en[ax] = nbr;
              on = m.pec && m.pec[en[0] + (int64_t)m.nx * (en[1] + (int64_t)m.ny * en[2])];
            }
            if (!on) continue;
            const int t1 = ax == 0 ? 1 : 0, t2 = ax == 2 ? 1 : 2;
            const double c = -0.5 * m.s * (side ? 1.0 : -1.0);
            // int_face N_p dN_q/dx_j dS for the face's nodes p (on the face)
            auto face_int = [&](const int (&lp)[3], const int (&lq)[3], int j) -> double {
              if (lp[ax] != side) return 0.0;
              if (j == ax) return (lq[ax] ? 1.0 : -1.0) / m.h[ax] * m1(lp[t1], lq[t1], m.h[t1]) *
                                  m1(lp[t2], lq[t2], m.h[t2]);
              if (lq[ax] != side) return 0.0;
              const int o = j == t1 ? t2 : t1;
              return g1(lq[j]) * m1(lp[o], lq[o], m.h[o]);
            };
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              K[ax][j].x += c * face_int(la, lb, j);
              K[j][ax].x += c * face_int(lb, la, j);
            }
          }
        }
        // ABC quads of this element containing both nodes
        if (m.abc_mask) {
#pragma unroll
          for (int f = 0; f < 6; ++f) {
            if (!((m.abc_mask >> f) & 1)) continue;
            const int ax = f >> 1, side = f & 1;
            if (d[ax] != 0 || la[ax] != side) continue;
            if (ee[ax] != (side ? nel[ax] - 1 : 0)) continue;
            const int t1 = ax == 0 ? 1 : 0, t2 = ax == 2 ? 1 : 2;
            const double Mf = mm[t1] * mm[t2];
            const double Sf = kk[t1] * mm[t2] + mm[t1] * kk[t2];
            // j k0 Mf + (j / 2k0) Sf on the tangential diagonal entries
            const double2 add = make_double2(0.0, m.k0 * Mf + Sf / (2.0 * m.k0));
            K[t1][t1] = cadd(K[t1][t1], add);
            K[t2][t2] = cadd(K[t2][t2], add);
          }
        }
      }
  // plane conditions: the fixed components' rows and columns become those of
  // the identity (slot 13 is the diagonal block)
  {
    const int gb3[3] = {gi[0] + d[0], gi[1] + d[1], gi[2] + d[2]};
    const int ca = fixed_components(m, gi), cb = fixed_components(m, gb3);
    if (ca | cb) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          if (((ca >> i) & 1) || ((cb >> j) & 1))
            K[i][j] = make_double2(slot == 13 && i == j ? 1.0 : 0.0, 0.0);
    }
  }
  double2* o64 = val64 + pos * 9;
  float2* o32 = val32 + pos * 9;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      o64[3 * i + j] = K[i][j];
      o32[3 * i + j] = make_float2((float)K[i][j].x, (float)K[i][j].y);
    }
  if (slot == 13) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double2 inv = cinv(K[i][i]);
      dinv64[3 * (int64_t)a + i] = inv;
      dinv32[3 * (int64_t)a + i] = make_float2((float)inv.x, (float)inv.y);
    }
  }
}

// ------------------------------------------------------------------ RHS
// b_(a,c) = sum over ABC faces and their active quads containing node a of
//   int N_a [ j k0 H_c - (n x curl H_i)_c ] + (j/2k0) grad_t N_a . grad_t H_c
// for tangential c, with curl H_i = -j k0 d x H_i, grad_t H_c = -j k0 d_t H_c,
// by 2x2 Gauss points on each quad.
__global__ void k_rhs(MeshDev m, PatternDev p, int32_t nrhs, const femh_plane_wave* __restrict__ waves,
                      double2* __restrict__ b) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)p.nn * nrhs) return;
  const int32_t a = (int32_t)(t % p.nn);
  const int r = (int)(t / p.nn);
  const int64_t gx = m.nx + 1, gy = m.ny + 1;
  const int64_t g = p.node_grid[a];
  const int gi[3] = {(int)(g % gx), (int)((g / gx) % gy), (int)(g / (gx * gy))};
  const int nel[3] = {m.nx, m.ny, m.nz};
  double2 acc[3] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
  const femh_plane_wave w = waves[r];
  const double k0 = m.k0;
  const double gp[2] = {0.5 - 0.5 / 1.7320508075688772935, 0.5 + 0.5 / 1.7320508075688772935};
  for (int f = 0; f < 6; ++f) {
    if (!((m.abc_mask >> f) & 1)) continue;
    const int ax = f >> 1, side = f & 1;
    if (gi[ax] != (side ? nel[ax] : 0)) continue;
    const int t1 = ax == 0 ? 1 : 0, t2 = ax == 2 ? 1 : 2;
    const double sgn = side ? 1.0 : -1.0;
    const double wq = 0.25 * m.h[t1] * m.h[t2];
    for (int e2 = gi[t2] - 1; e2 <= gi[t2]; ++e2) {
      if (e2 < 0 || e2 >= nel[t2]) continue;
      for (int e1 = gi[t1] - 1; e1 <= gi[t1]; ++e1) {
        if (e1 < 0 || e1 >= nel[t1]) continue;
        int ee[3];
        ee[ax] = side ? nel[ax] - 1 : 0;
        ee[t1] = e1;
        ee[t2] = e2;
        if (m.pec && m.pec[ee[0] + (int64_t)m.nx * (ee[1] + (int64_t)m.ny * ee[2])]) continue;
        const int l1 = gi[t1] - e1, l2 = gi[t2] - e2;
        for (int q2 = 0; q2 < 2; ++q2)
          for (int q1 = 0; q1 < 2; ++q1) {
            const double s1 = gp[q1], s2 = gp[q2];
            double rpos[3];
            rpos[ax] = m.origin[ax] + (ee[ax] + side) * m.h[ax];
            rpos[t1] = m.origin[t1] + (e1 + s1) * m.h[t1];
            rpos[t2] = m.origin[t2] + (e2 + s2) * m.h[t2];
            const double f1 = l1 ? s1 : 1.0 - s1, f2 = l2 ? s2 : 1.0 - s2;
            const double N = f1 * f2;
            const double dN1 = (l1 ? 1.0 : -1.0) / m.h[t1] * f2;
            const double dN2 = f1 * (l2 ? 1.0 : -1.0) / m.h[t2];
            const double phase = -k0 * (w.d[0] * rpos[0] + w.d[1] * rpos[1] + w.d[2] * rpos[2]);
            double sn, cs;
            sincos(phase, &sn, &cs);
            const double2 ex = make_double2(cs, sn);
            double2 H[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) H[c] = cmul(make_double2(w.p[c].re, w.p[c].im), ex);
            const double2 nH = cscale(H[ax], sgn);
            const double nd = sgn * w.d[ax];
            const double gNd = dN1 * w.d[t1] + dN2 * w.d[t2];
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {
              const int c = cc ? t2 : t1;
              // (n x curl H_i)_c = -j k0 (d_c (n.H) - H_c (n.d))
              const double2 inner = make_double2(w.d[c] * nH.x - H[c].x * nd, w.d[c] * nH.y - H[c].y * nd);
              const double2 ncurl = make_double2(k0 * inner.y, -k0 * inner.x);
              // j k0 H_c - ncurl
              const double2 jkH = make_double2(-k0 * H[c].y, k0 * H[c].x);
              double2 term = cscale(make_double2(jkH.x - ncurl.x, jkH.y - ncurl.y), N);
              // (j/2k0)(-j k0) H_c (grad_t N . d_t) = 0.5 H_c gNd
              term = cadd(term, cscale(H[c], 0.5 * gNd));
              acc[c] = cadd(acc[c], cscale(term, wq));
            }
          }
      }
    }
  }
  const int ca = fixed_components(m, gi);
#pragma unroll
  for (int c = 0; c < 3; ++c)
    if ((ca >> c) & 1) acc[c] = make_double2(0.0, 0.0);
  double2* out = b + (int64_t)r * 3 * p.nn + 3 * (int64_t)a;
  out[0] = acc[0];
  out[1] = acc[1];
  out[2] = acc[2];
}

// --------------------------------------------------------------- scatter
__global__ void k_scatter(int64_t ngrid, int32_t nn, int32_t nrhs, const int32_t* __restrict__ node_id,
                          const double2* __restrict__ x, double2* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ngrid * nrhs) return;
  const int64_t g = t % ngrid;
  const int64_t r = t / ngrid;
  const int32_t id = node_id[g];
  double2* o = out + (r * ngrid + g) * 3;
  if (id >= 0) {
    const double2* s = x + r * 3 * (int64_t)nn + 3 * (int64_t)id;
    o[0] = s[0];
    o[1] = s[1];
    o[2] = s[2];
  } else {
    o[0] = o[1] = o[2] = make_double2(0.0, 0.0);
  }
}

__global__ void k_copy_probe(const float4* __restrict__ src, float4* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ------------------------------------------------------ imported matrices
// complex64 copy of imported complex128 values (round to nearest, as the
// assembly writes it)
__global__ void k_round_c64(int64_t n, const double2* __restrict__ v64, float2* __restrict__ v32) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double2 v = v64[t];
  v32[t] = make_float2((float)v.x, (float)v.y);
}

// Jacobi inverse from an imported matrix's diagonal blocks: row a's block
// with column a (the host checked that it exists); bad gets 1 when a
// diagonal entry is zero
__global__ void k_dinv_from_blocks(int32_t nn, const int32_t* __restrict__ row_ptr,
                                   const int32_t* __restrict__ col_idx, const double2* __restrict__ val64,
                                   double2* __restrict__ dinv64, float2* __restrict__ dinv32,
                                   int32_t* __restrict__ bad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * (int64_t)nn) return;
  const int32_t a = (int32_t)(t / 3);
  const int i = (int)(t % 3);
  int32_t k = row_ptr[a];
  while (k < row_ptr[a + 1] - 1 && col_idx[k] != a) ++k;
  const double2 d = val64[(int64_t)k * 9 + 4 * i];
  if (d.x == 0.0 && d.y == 0.0) {
    *bad = 1;
    dinv64[t] = make_double2(0.0, 0.0);
    dinv32[t] = make_float2(0.f, 0.f);
    return;
  }
  const double2 inv = cinv(d);
  dinv64[t] = inv;
  dinv32[t] = make_float2((float)inv.x, (float)inv.y);
}

}  // namespace

namespace k {

hipError_t round_c64(hipStream_t st, int64_t n, const double2* v64, float2* v32) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_round_c64, dim3(grid_for(n, 256)), dim3(256), 0, st, n, v64, v32);
  return hipGetLastError();
}

hipError_t dinv_from_blocks(hipStream_t st, int32_t nn, const int32_t* row_ptr, const int32_t* col_idx,
                            const double2* val64, double2* dinv64, float2* dinv32, int32_t* bad) {
  const int64_t n = 3 * (int64_t)nn;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_dinv_from_blocks, dim3(grid_for(n, 256)), dim3(256), 0, st, nn, row_ptr, col_idx, val64,
                     dinv64, dinv32, bad);
  return hipGetLastError();
}


int64_t scan_tmp_ints(int64_t n) {
  int64_t total = 0;
  while (true) {
    int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles <= 0) tiles = 1;
    total += 2 * tiles;  // tile sums and their scan
    if (tiles <= 1) break;
    n = tiles;
  }
  return total + 8;
}

static hipError_t scan_rec(hipStream_t st, const int32_t* in, int32_t* out, int64_t n, int32_t* tmp) {
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  if (tiles == 0) return hipSuccess;
  int32_t* sums = tmp;
  int32_t* sums_scan = tmp + tiles;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(kScanThreads), 0, st, in, out, n, sums);
  if (tiles == 1) return hipGetLastError();
  hipError_t e = scan_rec(st, sums, sums_scan, tiles, tmp + 2 * tiles);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)tiles), dim3(256), 0, st, out, n, (const int32_t*)sums_scan);
  return hipGetLastError();
}

hipError_t exclusive_scan(hipStream_t st, const int32_t* in, int32_t* out, int64_t n, int32_t* tmp,
                          int32_t* total) {
  hipError_t e = scan_rec(st, in, out, n, tmp);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(64), 0, st, in, (const int32_t*)out, n, total);
  return hipGetLastError();
}

hipError_t check_materials(hipStream_t st, const double2* eps, const double2* mu, int64_t ne, int32_t* flag) {
  if (ne == 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_materials, dim3(grid_for(ne, 256)), dim3(256), 0, st, eps, mu, ne, flag);
  return hipGetLastError();
}

hipError_t node_flags(hipStream_t st, const MeshDev& m, int32_t* flags) {
  const int64_t n = (int64_t)(m.nx + 1) * (m.ny + 1) * (m.nz + 1);
  hipLaunchKernelGGL(k_node_flags, dim3(grid_for(n, 256)), dim3(256), 0, st, m, flags);
  return hipGetLastError();
}

hipError_t node_compact(hipStream_t st, const MeshDev& m, const int32_t* flags, const int32_t* scan,
                        int32_t* node_id, int32_t* node_grid) {
  const int64_t n = (int64_t)(m.nx + 1) * (m.ny + 1) * (m.nz + 1);
  hipLaunchKernelGGL(k_node_compact, dim3(grid_for(n, 256)), dim3(256), 0, st, n, flags, scan, node_id, node_grid);
  return hipGetLastError();
}

hipError_t row_masks(hipStream_t st, const MeshDev& m, int32_t nn, const int32_t* node_id,
                     const int32_t* node_grid, uint32_t* mask, int32_t* counts) {
  (void)node_id;
  if (nn == 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_masks, dim3(grid_for(nn, 256)), dim3(256), 0, st, m, nn, node_grid, mask, counts);
  return hipGetLastError();
}

hipError_t assemble(hipStream_t st, const MeshDev& m, const PatternDev& p, int32_t* col_idx, double2* val64,
                    float2* val32, double2* dinv64, float2* dinv32) {
  if (p.nn == 0) return hipSuccess;
  const int64_t threads = (int64_t)p.nn * 32;
  hipLaunchKernelGGL(k_assemble, dim3(grid_for(threads, 256)), dim3(256), 0, st, m, p, col_idx, val64, val32,
                     dinv64, dinv32);
  return hipGetLastError();
}

hipError_t rhs(hipStream_t st, const MeshDev& m, const PatternDev& p, int32_t nrhs, const femh_plane_wave* waves,
               double2* b) {
  const int64_t n = (int64_t)p.nn * nrhs;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rhs, dim3(grid_for(n, 128)), dim3(128), 0, st, m, p, nrhs, waves, b);
  return hipGetLastError();
}

hipError_t scatter(hipStream_t st, const MeshDev& m, const PatternDev& p, int32_t nrhs, const double2* x,
                   double2* out) {
  const int64_t ngrid = (int64_t)(m.nx + 1) * (m.ny + 1) * (m.nz + 1);
  const int64_t n = ngrid * nrhs;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(n, 256)), dim3(256), 0, st, ngrid, p.nn, nrhs, p.node_id, x, out);
  return hipGetLastError();
}

hipError_t copy_probe(hipStream_t st, const float4* src, float4* dst, int64_t n) {
  hipLaunchKernelGGL(k_copy_probe, dim3(256 * 16), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

}  // namespace k
}  // namespace femh
