// gfx950 kernels of the directional H2 compression (FP64 path).
//
// Block rows are processed by wave-level pipelines.  The operand of a wave
// is the weighted block row G^w_tc (leaf clusters: entries generated from
// the points; other clusters: the rows of G_hat_tc = zeta [R_t1c' ; R_t2c']
// read from the sons' coefficient matrices).  Consumers:
//   * Gram:      M += A A^*   (FP64 MFMA 16x16x4, lower-triangular tiles)
//   * R-product: R^T += A^T conj(Q)   (FP64 MFMA), i.e. R_tc = Q^* A
// The small factorisation (pivoted Cholesky of M, one-sided Jacobi on the
// factor) produces the left singular vectors and singular values of the block
// row (Section 6: the basis is formed by the first k left singular vectors).
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>
#include <utility>

#include <cmath>
#include <cstdint>

#include "common.hpp"
#include "kernels.hpp"

namespace dh2 {

typedef double dvec4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dvec4 mfma_f64(double a, double b, dvec4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Output layout of the FP64 16x16x4 MFMA (measured on gfx950): accumulator
// register v of lane l holds row (l / 16) + 4 v, column l % 16.  Operand A
// (16 x 4): lane l holds A[l % 16][l / 16]; operand B (4 x 16): B[l / 16][l % 16].
__device__ __forceinline__ int f64_row(int lane, int v) { return (lane >> 4) + 4 * v; }

typedef float fvec4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ fvec4 mfma_f32(float a, float b, fvec4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Output layout of the FP32 16x16x4 MFMA (measured on gfx950): register v of
// lane l holds row 4 (l / 16) + v, column l % 16; operands as for FP64.
__device__ __forceinline__ int f32_row(int lane, int v) { return 4 * (lane >> 4) + v; }

// Index of the calling wave in its workgroup as a wave-uniform value, so that
// loops and loads that depend only on it stay scalar.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// complex element of an R^T array stored in FP64 (MX false) or FP32 (MX true)
template <bool MX>
__device__ __forceinline__ double2 rload(const void* R, int64_t idx) {
  if constexpr (MX) {
    float2 v = reinterpret_cast<const float2*>(R)[idx];
    return make_double2(v.x, v.y);
  } else {
    return reinterpret_cast<const double2*>(R)[idx];
  }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Stored coupling matrices and near-field blocks: complex FP64 in the FP64
// form, complex FP32 in the mixed form (SE); arithmetic on them is FP64.
__device__ __forceinline__ double2 wide(double2 v) { return v; }
__device__ __forceinline__ double2 wide(float2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ void put(double2* p, int64_t i, double2 v) { p[i] = v; }
__device__ __forceinline__ void put(float2* p, int64_t i, double2 v) {
  p[i] = make_float2((float)v.x, (float)v.y);
}

// LDS written by some lanes of a wave and then read by others of the same
// wave: the writes complete and become visible before the reads
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr double kInv4Pi = 0.07957747154594767;  // 1/(4 pi)

// ---------------------------------------------------------------------------
// Matrix entries.  Side 0 reads G, side 1 reads G^* (rows of G^* are columns
// of G): entry(i,j) = conj(G_ji).
// ---------------------------------------------------------------------------
// sin and cos of x in [0, 2^20 pi/2): Cody-Waite reduction y = x - n pi/2
// with pi/2 split in three parts (the first two with 33 significant bits, so
// n * part is exact), then Taylor polynomials of sin and cos on |y| <= pi/4
// up to degree 17 and 16 (truncation error below 1e-18).
__device__ __forceinline__ void sincos_cw(double x, double& s, double& c) {
  double n = rint(x * 0.6366197723675814);
  double y = fma(-n, 0x1.921fb544p+0, x);
  y = fma(-n, 0x1.0b4611a6p-34, y);
  y = fma(-n, 0x1.3198a2e037073p-69, y);
  double y2 = y * y;
  double ps = 2.8114572543455206e-15;            // 1/17!
  ps = fma(ps, y2, -7.647163731819816e-13);       // -1/15!
  ps = fma(ps, y2, 1.6059043836821613e-10);       // 1/13!
  ps = fma(ps, y2, -2.505210838544172e-08);       // -1/11!
  ps = fma(ps, y2, 2.7557319223985893e-06);       // 1/9!
  ps = fma(ps, y2, -0.0001984126984126984);       // -1/7!
  ps = fma(ps, y2, 0.008333333333333333);         // 1/5!
  ps = fma(ps, y2, -0.16666666666666666);         // -1/3!
  double sy = fma(ps * y2, y, y);
  double pc = 4.779477332387385e-14;             // 1/16!
  pc = fma(pc, y2, -1.1470745597729725e-11);      // -1/14!
  pc = fma(pc, y2, 2.08767569878681e-09);         // 1/12!
  pc = fma(pc, y2, -2.755731922398589e-07);       // -1/10!
  pc = fma(pc, y2, 2.48015873015873e-05);         // 1/8!
  pc = fma(pc, y2, -0.001388888888888889);        // -1/6!
  pc = fma(pc, y2, 0.041666666666666664);         // 1/4!
  pc = fma(pc, y2, -0.5);                         // -1/2!
  double cy = fma(pc, y2, 1.0);
  int q = (int)((long long)n & 3);
  double ss = (q & 1) ? cy : sy, cc = (q & 1) ? sy : cy;
  s = (q & 2) ? -ss : ss;
  c = ((q + 1) & 2) ? -cc : cc;
}

__device__ __forceinline__ void sincos_phase(double x, double& s, double& c) {
  if (x < 1.6e6)
    sincos_cw(x, s, c);
  else
    sincos(x, &s, &c);
}

// Mixed precision: the same Cody-Waite reduction in FP64 (two parts suffice
// at FP32 accuracy), then Taylor polynomials of degree 11/10 in FP32
// (truncation below 1e-10 on |y| <= pi/4).
__device__ __forceinline__ void sincos_mixed(double x, float& s, float& c) {
  double n = rint(x * 0.6366197723675814);
  double y = fma(-n, 0x1.921fb544p+0, x);
  y = fma(-n, 0x1.0b4611a6p-34, y);
  float yf = (float)y;
  float y2 = yf * yf;
  float ps = -2.5052108e-08f;                // -1/11!
  ps = fmaf(ps, y2, 2.7557319e-06f);          // 1/9!
  ps = fmaf(ps, y2, -1.9841270e-04f);         // -1/7!
  ps = fmaf(ps, y2, 8.3333333e-03f);          // 1/5!
  ps = fmaf(ps, y2, -1.6666667e-01f);         // -1/3!
  float sy = fmaf(ps * y2, yf, yf);
  float pc = -2.7557319e-07f;                // -1/10!
  pc = fmaf(pc, y2, 2.4801587e-05f);          // 1/8!
  pc = fmaf(pc, y2, -1.3888889e-03f);         // -1/6!
  pc = fmaf(pc, y2, 4.1666667e-02f);          // 1/4!
  pc = fmaf(pc, y2, -0.5f);                   // -1/2!
  float cy = fmaf(pc, y2, 1.0f);
  int q = (int)n & 3;  // |n| < 2^31 for the phases that occur
  float ss = (q & 1) ? cy : sy, cc = (q & 1) ? sy : cy;
  s = (q & 2) ? -ss : ss;
  c = ((q + 1) & 2) ? -cc : cc;
}

// 1/sqrt(r2) to about half an ulp: hardware estimate refined by one Newton
// step whose residual is formed with an FMA.
__device__ __forceinline__ double rsqrt_nr(double r2) {
  double ri = rsqrt(r2);
  double h = r2 * ri;                 // ~ sqrt(r2)
  double e = fma(-h, ri, 1.0);        // 1 - r2 ri^2
  return fma(0.5 * ri, e, ri);
}

// w exp(+-i kappa r) / (4 pi r) from the difference vector (r > 0)
__device__ __forceinline__ double2 helm_offdiag(double dx, double dy, double dz, double w,
                                                double kappa, int side) {
  double r2 = dx * dx + dy * dy + dz * dz;
  double ri = rsqrt_nr(r2);
  double r = r2 * ri;
  double s, c;
  sincos_phase(kappa * r, s, c);
  double a = w * kInv4Pi * ri;
  return make_double2(a * c, side == 0 ? a * s : -a * s);
}

__device__ __forceinline__ double2 helm_entry(const GeomDev& g, int64_t pi, int64_t pj, int side) {
  const double* xi = g.pts + 4 * pi;
  const double* xj = g.pts + 4 * pj;
  if (pi == pj) {
    double w = xi[3];
    double im = g.kappa * w * kInv4Pi;
    return make_double2(0.5 * sqrt(w * 0.3183098861837907), side == 0 ? im : -im);
  }
  double w = side == 0 ? xj[3] : xi[3];
  return helm_offdiag(xi[0] - xj[0], xi[1] - xj[1], xi[2] - xj[2], w, g.kappa, side);
}

__device__ __forceinline__ double2 dense_entry(const GeomDev& g, int64_t pi, int64_t pj, int side) {
  const double2* G = reinterpret_cast<const double2*>(g.G);
  if (side == 0) return G[g.perm[pi] * g.ldg + g.perm[pj]];
  double2 v = G[g.perm[pj] * g.ldg + g.perm[pi]];
  return make_double2(v.x, -v.y);
}

// Double layer (Section 7, DLP matrix, collocation form): the entry of G at
// (x point p, y point q) is w_q (1 - i kappa r) exp(i kappa r)
// <x_p - x_q, n_q> / (4 pi r^3), and 1/2 on the diagonal; G^* (side 1) takes
// the row as the y point and conjugates.
__device__ __forceinline__ double2 dlp_entry(const GeomDev& g, int64_t pi, int64_t pj, int side) {
  if (pi == pj) return make_double2(0.5, 0.0);
  const int64_t p = side == 0 ? pi : pj, q = side == 0 ? pj : pi;
  const double* xp = g.pts + 4 * p;
  const double* xq = g.pts + 4 * q;
  const double* nq = g.nrm + 4 * q;
  double dx = xp[0] - xq[0], dy = xp[1] - xq[1], dz = xp[2] - xq[2];
  double r2 = dx * dx + dy * dy + dz * dz;
  double ri = rsqrt_nr(r2);
  double r = r2 * ri;
  double s, c;
  sincos_phase(g.kappa * r, s, c);
  // (1 - i kappa r)(c + i s) = (c + kappa r s) + i (s - kappa r c)
  double kr = g.kappa * r;
  double a = xq[3] * kInv4Pi * (dx * nq[0] + dy * nq[1] + dz * nq[2]) * ri * ri * ri;
  double re = a * (c + kr * s), im = a * (s - kr * c);
  return make_double2(re, side == 0 ? im : -im);
}

template <int SRC>
__device__ __forceinline__ double2 entry(const GeomDev& g, int64_t pi, int64_t pj, int side) {
  if constexpr (SRC == SRC_HELMHOLTZ)
    return helm_entry(g, pi, pj, side);
  else if constexpr (SRC == SRC_DLP)
    return dlp_entry(g, pi, pj, side);
  else
    return dense_entry(g, pi, pj, side);
}

// ---------------------------------------------------------------------------
// Block norms: omega_b^2 = sum |G_ij|^2 over the admissible block.
// ---------------------------------------------------------------------------
template <int SRC>
__global__ __launch_bounds__(256) void k_block_norm(GeomDev g, const int64_t* t_off,
                                                    const int64_t* t_len, const int64_t* s_off,
                                                    const int64_t* s_len, int64_t nblocks,
                                                    double* omega) {
  __shared__ double red[256];
  int64_t b = blockIdx.x;
  if (b >= nblocks) return;
  const int64_t to = t_off[b], tl = t_len[b], so = s_off[b], sl = s_len[b];
  // four row groups x 64 column lanes
  const int ty = wave_id(), tx = threadIdx.x & 63;
  double acc = 0.0;
  if constexpr (SRC == SRC_HELMHOLTZ) {
    // the lane keeps its column point in registers; the wave's rows are
    // wave-uniform (scalar loads); 1/r^2 is the hardware reciprocal refined
    // by two Newton steps
    for (int64_t j = so + tx; j < so + sl; j += 64) {
      const double* xj = g.pts + 4 * j;
      const double y0 = xj[0], y1 = xj[1], y2 = xj[2];
      const double a = xj[3] * kInv4Pi, a2 = a * a;
#pragma unroll 4
      for (int64_t i = to + ty; i < to + tl; i += 4) {
        const double* xi = g.pts + 4 * i;
        double dx = xi[0] - y0, dy = xi[1] - y1, dz = xi[2] - y2;
        double r2 = dx * dx + dy * dy + dz * dz;
        double q = __builtin_amdgcn_rcp(r2);
        q = fma(q, fma(-r2, q, 1.0), q);
        q = fma(q, fma(-r2, q, 1.0), q);
        acc = fma(a2, q, acc);
      }
    }
  } else {
    for (int64_t i = to + ty; i < to + tl; i += 4)
      for (int64_t j = so + tx; j < so + sl; j += 64) {
        double2 z = entry<SRC>(g, i, j, 0);
        acc += z.x * z.x + z.y * z.y;
      }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) omega[b] = sqrt(red[0]);
}

// Spectral block norms: omega_b = ||G|_b||_2 by the power method on
// (G|_b)^* G|_b, one workgroup per block, entries generated in every pass.
// With x normalised, ||G|_b x||^2 increases to sigma_1^2; the iteration
// stops when it changes by less than tol (relative) or after max_iter steps.
constexpr int kNorm2Max = 1024;  // largest cluster of an admissible block
__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

template <int SRC>
__global__ __launch_bounds__(256) void k_block_norm2(GeomDev g, const int64_t* t_off,
                                                     const int64_t* t_len, const int64_t* s_off,
                                                     const int64_t* s_len, int64_t nblocks,
                                                     int max_iter, double tol, double* omega) {
  __shared__ double2 xs[kNorm2Max];
  __shared__ double2 ys[kNorm2Max];
  __shared__ double red[4];
  const int64_t b = blockIdx.x;
  if (b >= nblocks) return;
  const int64_t to = t_off[b], so = s_off[b];
  const int tl = (int)t_len[b], sl = (int)s_len[b];
  const int tid = threadIdx.x;
  // start vector with no special structure (fixed, so runs repeat exactly)
  double p = 0.0;
  for (int j = tid; j < sl; j += 256) {
    double2 v = make_double2(1.0 + 0.5 * sin(0.7 * j), 0.3 * cos(1.3 * j));
    xs[j] = v;
    p += v.x * v.x + v.y * v.y;
  }
  double nx = sqrt(block_sum(p, red));
  for (int j = tid; j < sl; j += 256) xs[j] = make_double2(xs[j].x / nx, xs[j].y / nx);
  __syncthreads();
  double lam = 0.0;
  for (int it = 0; it < max_iter; ++it) {
    // y = G|_b x
    p = 0.0;
    for (int i = tid; i < tl; i += 256) {
      double2 acc = make_double2(0.0, 0.0);
      for (int j = 0; j < sl; ++j) {
        double2 a = entry<SRC>(g, to + i, so + j, 0), x = xs[j];
        acc.x += a.x * x.x - a.y * x.y;
        acc.y += a.x * x.y + a.y * x.x;
      }
      ys[i] = acc;
      p += acc.x * acc.x + acc.y * acc.y;
    }
    const double lam_new = block_sum(p, red);  // ||G|_b x||^2, x normalised
    // x = (G|_b)^* y, normalised
    p = 0.0;
    for (int j = tid; j < sl; j += 256) {
      double2 acc = make_double2(0.0, 0.0);
      for (int i = 0; i < tl; ++i) {
        double2 a = entry<SRC>(g, to + i, so + j, 0), y = ys[i];
        acc.x += a.x * y.x + a.y * y.y;  // conj(a) y
        acc.y += a.x * y.y - a.y * y.x;
      }
      xs[j] = acc;
      p += acc.x * acc.x + acc.y * acc.y;
    }
    nx = sqrt(block_sum(p, red));
    const bool done = !(nx > 0.0) || fabs(lam_new - lam) <= tol * lam_new;
    lam = lam_new;
    if (done) break;
    for (int j = tid; j < sl; j += 256) xs[j] = make_double2(xs[j].x / nx, xs[j].y / nx);
    __syncthreads();
  }
  if (tid == 0) omega[b] = sqrt(lam);
}

// scale of each column-set entry: 1 / (omega_b zeta^d)
__global__ void k_entry_scale(EntDev* ent, int64_t nent, const double* omega, double zeta) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nent) return;
  double z = 1.0;
  for (int q = 0; q < ent[e].d; ++q) z *= zeta;
  ent[e].scale = 1.0 / (omega[ent[e].b] * z);
}

__device__ __forceinline__ void pair_ij(int p, int& I, int& J) {
  I = 0;
  while ((I + 1) * (I + 2) / 2 <= p) ++I;
  J = p - I * (I + 1) / 2;
}

// Sum the partial Grams of each item (in unit order) into M (r x r,
// column-major, Hermitian: both triangles written).
__global__ __launch_bounds__(256) void k_gram_reduce(const ItemDev* items, const int32_t* litems,
                                                     const int32_t* ubegin, const UnitDev* units,
                                                     const double2* partial) {
  int32_t i = litems[blockIdx.x];
  const ItemDev& it = items[i];
  int r = it.r, nt = (r + 15) / 16, npairs = nt * (nt + 1) / 2;
  int32_t ub = ubegin[blockIdx.x], ue = ubegin[blockIdx.x + 1];
  double2* Mi = it.M;
  for (int e = threadIdx.x; e < npairs * 256; e += 256) {
    double2 s = make_double2(0.0, 0.0);
    int p = e >> 8, v = (e >> 6) & 3, lane = e & 63;
    int I, J;
    pair_ij(p, I, J);
    for (int32_t q = ub; q < ue; ++q) {
      const UnitDev& uq = units[q];
      int loc;
      if (uq.a0 == uq.b0) {  // diagonal block of tiles
        if (I < uq.a0 || I >= uq.a0 + uq.na || J < uq.b0) continue;
        int Il = I - uq.a0, Jl = J - uq.b0;
        loc = Il * (Il + 1) / 2 + Jl;
      } else {
        if (I < uq.a0 || I >= uq.a0 + uq.na || J < uq.b0 || J >= uq.b0 + uq.nb) continue;
        loc = (I - uq.a0) * uq.nb + (J - uq.b0);
      }
      double2 val = partial[uq.slot_off + (int64_t)loc * 256 + (e & 255)];
      s.x += val.x;
      s.y += val.y;
    }
    int row = 16 * I + f64_row(lane, v), col = 16 * J + (lane & 15);
    if (row < r && col < r) {
      if (I != J || row >= col) {
        Mi[row + (int64_t)col * r] = s;
        if (row != col) Mi[col + (int64_t)row * r] = make_double2(s.x, -s.y);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Factorisation of one Gram matrix: pivoted Cholesky M ~ X X^* (stopped when
// the remaining diagonal falls below tau), then one-sided Jacobi on X.
// The columns of the rotated X are U Sigma: U = left singular vectors of the
// block row, Sigma its singular values.  Output: sigma (descending, r values,
// zeros past the factor), Q = first k columns of U (row-major r x k),
// k = #{sigma > eps}.
// ---------------------------------------------------------------------------
constexpr int kEigLds = 9216;  // largest X in double2 elements (144 KiB)
constexpr int kFacLdsX = 4800;  // X of the first pass (75 KiB: two workgroups per CU)
constexpr int kFacThreads = 256;
// dynamic LDS of the non-leaf R-product (160 KiB per CU minus its static LDS)
constexpr size_t kRprodLdsMax = 159 * 1024;

// 1/sqrt(x) and 1/x (x > 0, normal): the hardware estimates refined by two
// Newton steps with FMA residuals (each step squares the relative error)
__device__ __forceinline__ double rsq_nr2(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}
__device__ __forceinline__ double rcp_nr2(double x) {
  double y = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
  }
  return y;
}

__device__ __forceinline__ double wave_sum(double v, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// RMAX bounds r; GX: X in global memory (xptr[blockIdx.x], r (r + 1)
// elements) for factors too large for LDS, else in dynamic LDS.
template <int RMAX, bool GX>
__global__ __launch_bounds__(kFacThreads) void k_factor(ItemDev* items, const int32_t* litems,
                                                        double eps, int max_sweeps, int cap,
                                                        int32_t* status, double2* const* xptr) {
  extern __shared__ double2 Xs[];  // column-major r x pmax
  double2* X = GX ? xptr[blockIdx.x] : Xs;
  __shared__ double d[RMAX];
  __shared__ int done[RMAX];
  __shared__ double bval[4];
  __shared__ int bidx[4];
  __shared__ int s_piv;
  __shared__ double s_dmax;
  __shared__ int s_p;
  __shared__ int s_rot;
  __shared__ double s_norm[RMAX];
  __shared__ int s_rank[RMAX];

  int32_t ii = litems[blockIdx.x];
  ItemDev& it = items[ii];
  int r = it.r;
  int tid = threadIdx.x, lane = tid & 63, w = wave_id();
  const double2* Mi = it.M;
  if (r == 0) {
    if (tid == 0) it.k = 0;
    return;
  }
  // X holds ncap columns; the pairing needs an even column count pe <= ncap
  int ncap = cap / r;
  int pmax = r < ncap ? r : ncap;
  if ((pmax & 1) && pmax + 1 > ncap) --pmax;

  double dmax0 = 0.0;
  for (int i = tid; i < r; i += 256) {
    d[i] = Mi[i + (int64_t)i * r].x;
    done[i] = 0;
  }
  __syncthreads();
  for (int i = 0; i < r; ++i) dmax0 = fmax(dmax0, d[i]);
  double tau = fmax(1e-4 * eps * eps / r, 64.0 * 2.220446049250313e-16 * dmax0);

  // ---- pivoted Cholesky, left-looking ----
  int p = 0;
  for (int j = 0; j < pmax; ++j) {
    // argmax of d over rows not yet pivoted
    double bv = -1.0;
    int bi = -1;
    for (int i = tid; i < r; i += 256)
      if (!done[i] && d[i] > bv) {
        bv = d[i];
        bi = i;
      }
    for (int o = 32; o > 0; o >>= 1) {
      double ov = __shfl_xor(bv, o, 64);
      int oi = __shfl_xor(bi, o, 64);
      if (ov > bv || (ov == bv && oi >= 0 && (bi < 0 || oi < bi))) {
        bv = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      bval[w] = bv;
      bidx[w] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double v = bval[0];
      int ix = bidx[0];
      for (int q = 1; q < 4; ++q)
        if (bval[q] > v || (bval[q] == v && bidx[q] >= 0 && (ix < 0 || bidx[q] < ix))) {
          v = bval[q];
          ix = bidx[q];
        }
      s_piv = ix;
      s_dmax = v;
    }
    __syncthreads();
    int piv = s_piv;
    double dm = s_dmax;
    if (piv < 0 || !(dm > tau)) break;
    double sq = sqrt(dm), inv = 1.0 / sq;
    for (int i = tid; i < r; i += 256) {
      double2 v;
      if (i == piv) {
        v = make_double2(sq, 0.0);
      } else if (done[i]) {
        v = make_double2(0.0, 0.0);
      } else {
        double2 a = Mi[i + (int64_t)piv * r];
        for (int q = 0; q < j; ++q) {
          double2 x = X[q * r + i], y = X[q * r + piv];
          // a -= x * conj(y)
          a.x -= x.x * y.x + x.y * y.y;
          a.y -= x.y * y.x - x.x * y.y;
        }
        v = make_double2(a.x * inv, a.y * inv);
      }
      X[j * r + i] = v;
    }
    __syncthreads();
    for (int i = tid; i < r; i += 256) {
      if (i == piv) {
        done[i] = 1;
        d[i] = 0.0;
      } else if (!done[i]) {
        double2 v = X[j * r + i];
        d[i] = fmax(0.0, d[i] - (v.x * v.x + v.y * v.y));
      }
    }
    __syncthreads();
    p = j + 1;
  }
  if (tid == 0) {
    s_p = p;
    // the factorisation stopped at the column capacity while a remaining
    // diagonal entry still exceeds tau (the cut the factor would have taken
    // otherwise)
    double rest = 0.0;
    for (int i = 0; i < r; ++i)
      if (!done[i]) rest = fmax(rest, d[i]);
    s_rot = 0;
    if (p == pmax && rest > tau) {
      // X in memory holds all r columns, so this cannot happen there; the
      // LDS-resident kernel marks the item (rank -1) for the host to factor it
      // again with X in memory
      if (GX) atomicMax(status, 1);
      else s_rot = 1;
    }
  }
  __syncthreads();
  if (s_rot) {
    if (tid == 0) it.k = -1;
    return;
  }
  p = s_p;
  int pe = p + (p & 1);
  for (int i = tid; i < r; i += 256)
    if (pe > p) X[p * r + i] = make_double2(0.0, 0.0);
  __syncthreads();

  // ---- one-sided Jacobi on the columns of X (r x pe) ----
  int npair = pe / 2;
  int g = 1;
  while (g * 2 * npair <= 256 && g < 64) g *= 2;
  int pair = tid / g, gl = tid % g;
  int sweep = 0;
  if (pe >= 2) {
    for (sweep = 0; sweep < max_sweeps; ++sweep) {
      if (tid == 0) s_rot = 0;
      __syncthreads();
      for (int step = 0; step < pe - 1; ++step) {
        if (pair < npair) {
          int pa = pair, pb = pe - 1 - pair;
          int a = pa == 0 ? 0 : 1 + (pa - 1 + step) % (pe - 1);
          int b = pb == 0 ? 0 : 1 + (pb - 1 + step) % (pe - 1);
          // squared column norms: summed in the first step of a sweep (its
          // pairs cover every column), then carried through the rotations
          // (|x'|^2 = |x|^2 - t |<x, y>|, |y'|^2 = |y|^2 + t |<x, y>|)
          double al = 0, be = 0, gr = 0, gi = 0;
          if (step == 0) {
            for (int i = gl; i < r; i += g) {
              double2 x = X[a * r + i], y = X[b * r + i];
              al += x.x * x.x + x.y * x.y;
              be += y.x * y.x + y.y * y.y;
              gr += x.x * y.x + x.y * y.y;  // conj(x) * y
              gi += x.x * y.y - x.y * y.x;
            }
            al = wave_sum(al, g);
            be = wave_sum(be, g);
          } else {
            for (int i = gl; i < r; i += g) {
              double2 x = X[a * r + i], y = X[b * r + i];
              gr += x.x * y.x + x.y * y.y;
              gi += x.x * y.y - x.y * y.x;
            }
            al = s_norm[a];
            be = s_norm[b];
          }
          gr = wave_sum(gr, g);
          gi = wave_sum(gi, g);
          const double g2 = gr * gr + gi * gi;  // |<x, y>|^2
          // rotate unless |<x, y>| <= 1e-15 |x| |y|
          if (g2 > 1e-30 * al * be && g2 > 1e-280) {
            // rotation parameters from hardware reciprocal (square-root)
            // estimates refined by two Newton steps each (to the last bits;
            // c^2 + s^2 = 1 to rounding, so the rotation stays orthogonal)
            const double iag = rsq_nr2(g2);  // 1 / |<x, y>|
            double tz = (be - al) * 0.5 * iag;
            const double h = fma(tz, tz, 1.0);
            double t = rcp_nr2(fabs(tz) + h * rsq_nr2(h));
            if (tz < 0) t = -t;
            double c = rsq_nr2(fma(t, t, 1.0)), s = c * t;
            double er = gr * iag, ei = -gi * iag;  // e^{-i phi}
            for (int i = gl; i < r; i += g) {
              double2 x = X[a * r + i], y = X[b * r + i];
              double2 ey = make_double2(er * y.x - ei * y.y, er * y.y + ei * y.x);
              X[a * r + i] = make_double2(c * x.x - s * ey.x, c * x.y - s * ey.y);
              X[b * r + i] = make_double2(s * x.x + c * ey.x, s * x.y + c * ey.y);
            }
            const double tg = t * (g2 * iag);
            al = fmax(0.0, al - tg);
            be += tg;
            if (gl == 0) s_rot = 1;
          }
          // the pair's lanes are one wave: all have read the norms above
          if (gl == 0) {
            s_norm[a] = al;
            s_norm[b] = be;
          }
        }
        __syncthreads();
      }
      int rot = s_rot;
      __syncthreads();
      if (!rot) break;
    }
    if (sweep == max_sweeps && tid == 0) atomicMax(status, 2);
    if (tid == 0) {
      atomicAdd(status + 1, sweep + 1);
      atomicAdd(status + 2, 1);
    }
  }

  // ---- singular values, ordering, rank ----
  for (int q = tid; q < pe; q += 256) {
    double s2 = 0;
    for (int i = 0; i < r; ++i) {
      double2 x = X[q * r + i];
      s2 += x.x * x.x + x.y * x.y;
    }
    s_norm[q] = sqrt(s2);
  }
  __syncthreads();
  for (int q = tid; q < pe; q += 256) {
    int rk = 0;
    double v = s_norm[q];
    for (int q2 = 0; q2 < pe; ++q2) {
      double o = s_norm[q2];
      if (o > v || (o == v && q2 < q)) ++rk;
    }
    s_rank[q] = rk;
  }
  __syncthreads();
  int k = 0;
  for (int q = 0; q < pe; ++q)
    if (s_norm[q] > eps) ++k;
  double* sg = it.sig;
  for (int q = tid; q < r; q += 256) sg[q] = 0.0;
  __syncthreads();
  for (int q = tid; q < pe; q += 256)
    if (s_rank[q] < r) sg[s_rank[q]] = s_norm[q];  // the zero pad column may rank r
  double2* Q = it.Q;  // row-major r x k
  for (int e = tid; e < pe * r; e += 256) {
    int q = e / r, i = e - q * r;
    int rk = s_rank[q];
    if (rk < k) {
      double inv = 1.0 / s_norm[q];
      double2 x = X[q * r + i];
      Q[(int64_t)i * k + rk] = make_double2(x.x * inv, x.y * inv);
    }
  }
  if (tid == 0) it.k = k;
}

__global__ __launch_bounds__(256) void k_ranks(const ItemDev* items, int32_t n, int32_t* out) {
  int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = items[i].k;
}

// ---------------------------------------------------------------------------
// Expansion of the column basis: dst rows = src (rows x ks) * E (ks x k).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_expand(const ExpandDev* tasks) {
  const ExpandDev t = tasks[blockIdx.x];
  int64_t tot = (int64_t)t.rows * t.k;
  for (int64_t e = threadIdx.x; e < tot; e += 256) {
    int64_t i = e / t.k;
    int kk = (int)(e - i * t.k);
    double2 s = make_double2(0.0, 0.0);
    for (int q = 0; q < t.ks; ++q) {
      double2 a = t.src[i * t.ks + q];
      double2 b = t.E[(int64_t)q * t.k + kk];
      s.x += a.x * b.x - a.y * b.y;
      s.y += a.x * b.y + a.y * b.x;
    }
    t.dst[i * t.k + kk] = s;
  }
}

// mixed form: complex FP64 -> FP32 copies, one workgroup per task
__global__ __launch_bounds__(256) void k_cvt(const CvtDev* tasks) {
  const CvtDev t = tasks[blockIdx.x];
  for (int64_t e = threadIdx.x; e < t.count; e += 256)
    t.dst[e] = make_float2((float)t.src[e].x, (float)t.src[e].y);
}

// copy a leaf basis (row-major rows x k) into the expanded-basis arena
__global__ void k_copy_c(const double2* src, int64_t src_off, double2* dst, int64_t dst_off,
                         int64_t count) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) dst[dst_off + e] = src[src_off + e];
}

// ---------------------------------------------------------------------------
// Projection: S_b = omega_b (R_tc restricted to the columns of s) Wexp_sc,
// one wave per block; FP32 MFMA in the mixed form.
// ---------------------------------------------------------------------------
template <bool MX>
struct SAcc;
template <>
struct SAcc<false> {
  dvec4 re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
  __device__ __forceinline__ void mac(double2 a, double2 b) {  // a b
    re = mfma_f64(a.x, b.x, re);
    re = mfma_f64(-a.y, b.y, re);
    im = mfma_f64(a.x, b.y, im);
    im = mfma_f64(a.y, b.x, im);
  }
  __device__ __forceinline__ int row(int lane, int v) const { return f64_row(lane, v); }
  __device__ __forceinline__ double2 get(int v) const { return make_double2(re[v], im[v]); }
};
template <>
struct SAcc<true> {
  fvec4 re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
  __device__ __forceinline__ void mac(double2 a, double2 b) {
    float ar = (float)a.x, ai = (float)a.y, br = (float)b.x, bi = (float)b.y;
    re = mfma_f32(ar, br, re);
    re = mfma_f32(-ai, bi, re);
    im = mfma_f32(ar, bi, im);
    im = mfma_f32(ai, br, im);
  }
  __device__ __forceinline__ int row(int lane, int v) const { return f32_row(lane, v); }
  __device__ __forceinline__ double2 get(int v) const { return make_double2(re[v], im[v]); }
};

template <bool MX>
__global__ __launch_bounds__(256) void k_project(const ProjDev* tasks, int64_t ntasks,
                                                 const double* omega) {
  int64_t ti = (int64_t)blockIdx.x * 4 + wave_id();
  if (ti >= ntasks) return;
  const ProjDev t = tasks[ti];
  int lane = threadIdx.x & 63, row = lane & 15, kq = lane >> 4;
  int kt = t.kt, ks = t.ks;
  if (kt == 0 || ks == 0) return;
  double om = omega[t.b];
  int nti = (kt + 15) / 16, ntj = (ks + 15) / 16;
  const void* Wb = t.W;
  using SE = typename std::conditional<MX, float2, double2>::type;
  SE* Sb = static_cast<SE*>(t.S);
  // column tiles of S in groups of eight (ranks beyond 128 take several)
  for (int tj0 = 0; tj0 < ntj; tj0 += 8)
  for (int ti16 = 0; ti16 < nti; ++ti16) {
    SAcc<MX> acc[8];
    int ii = ti16 * 16 + row;
    for (int j0 = 0; j0 < t.ns; j0 += 4) {
      int j = j0 + kq;
      double2 a = (j < t.ns && ii < kt) ? rload<MX>(t.R, (int64_t)j * kt + ii) : make_double2(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (tj0 + q < ntj) {
          int jj = (tj0 + q) * 16 + row;
          double2 b = (j < t.ns && jj < ks) ? rload<MX>(Wb, (int64_t)j * ks + jj) : make_double2(0.0, 0.0);
          acc[q].mac(a, b);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (tj0 + q < ntj) {
        int jj = (tj0 + q) * 16 + row;
        for (int v = 0; v < 4; ++v) {
          int i = ti16 * 16 + acc[q].row(lane, v);
          double2 z = acc[q].get(v);
          if (i < kt && jj < ks) put(Sb, i + (int64_t)jj * kt, make_double2(om * z.x, om * z.y));
        }
      }
    }
  }
}

// Tiled projection for blocks with ks <= 64: one wave per (block, pass over
// NI row tiles), all NI x NJ tile pairs accumulated in registers over one
// sweep of the columns of s, operands loaded one k-step ahead.  Workgroups
// are mapped so that the workgroups on one XCD take a contiguous range of
// the (W-sorted) task list and share the expanded bases in their L2.
template <bool MX>
struct POp;
template <>
struct POp<false> {
  double re, im;
};
template <>
struct POp<true> {
  float re, im;
};

// Load of element idx of a complex array in device memory, through a global
// (not flat) pointer so that only the vector memory counter tracks it.
// Buffer resource over the first `bytes` bytes at p (raw addressing, no
// stride).  Loads through it at byte offsets past `bytes` return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

// Complex element at byte offset off of a buffer (zero past its end).
template <bool MX>
__device__ __forceinline__ POp<MX> pload(__amdgpu_buffer_rsrc_t r, int off) {
  if constexpr (MX) {
    typedef float E __attribute__((ext_vector_type(2)));
    E v = __builtin_bit_cast(E, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    return POp<MX>{v.x, v.y};
  } else {
    typedef double E __attribute__((ext_vector_type(2)));
    E v = __builtin_bit_cast(E, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    return POp<MX>{v.x, v.y};
  }
}

template <bool MX>
struct PAcc;
template <>
struct PAcc<false> {
  dvec4 re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
  // acc += a b (complex)
  __device__ __forceinline__ void mac(const POp<false>& a, const POp<false>& b) {
    re = mfma_f64(a.re, b.re, re);
    re = mfma_f64(-a.im, b.im, re);
    im = mfma_f64(a.re, b.im, im);
    im = mfma_f64(a.im, b.re, im);
  }
  __device__ __forceinline__ int row(int lane, int v) const { return f64_row(lane, v); }
  __device__ __forceinline__ double2 get(int v) const { return make_double2(re[v], im[v]); }
};
template <>
struct PAcc<true> {
  fvec4 re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
  __device__ __forceinline__ void mac(const POp<true>& a, const POp<true>& b) {
    re = mfma_f32(a.re, b.re, re);
    re = mfma_f32(-a.im, b.im, re);
    im = mfma_f32(a.re, b.im, im);
    im = mfma_f32(a.im, b.re, im);
  }
  __device__ __forceinline__ int row(int lane, int v) const { return f32_row(lane, v); }
  __device__ __forceinline__ double2 get(int v) const { return make_double2(re[v], im[v]); }
};

// Accumulates the NI x NJ tile pairs of row tiles ti0.. over columns
// [jb, je) of s (jb a multiple of 4, jb < je).  Every load is unconditional:
// row and column indices past kt, ks only feed accumulator rows and columns
// that are never stored, so they are clamped to the last valid one; columns
// of s past je lie outside the buffer ranges and load as zero.  Operands are
// loaded three k-steps ahead into a ring of four register sets that is
// unrolled, so no loaded register is copied (a copy would wait for the load).
template <bool MX, int NI, int NJ>
__device__ void proj_acc(const ProjDev& t, int ti0, int jb, int je, PAcc<MX> (&acc)[NI][NJ]) {
  int lane = threadIdx.x & 63, row = lane & 15, kq = lane >> 4;
  const int kt = t.kt, ks = t.ks;
  constexpr int esz = sizeof(POp<MX>);
  // columns of s past je read as zero from both buffers
  const __amdgpu_buffer_rsrc_t rR = buf_rsrc(t.R, (int64_t)je * kt * esz);
  const __amdgpu_buffer_rsrc_t rW = buf_rsrc(t.W, (int64_t)je * ks * esz);
  int ra[NI], wa[NJ];
#pragma unroll
  for (int I = 0; I < NI; ++I) ra[I] = min(16 * (ti0 + I) + row, kt - 1) * esz;
#pragma unroll
  for (int J = 0; J < NJ; ++J) wa[J] = min(16 * J + row, ks - 1) * esz;
  auto load = [&](int j, POp<MX>* aa, POp<MX>* bb) {
#pragma unroll
    for (int I = 0; I < NI; ++I) aa[I] = pload<MX>(rR, j * kt * esz + ra[I]);
#pragma unroll
    for (int J = 0; J < NJ; ++J) bb[J] = pload<MX>(rW, j * ks * esz + wa[J]);
  };
  // accumulators hold S^T tiles (rows: columns of W, columns: rows of R^T),
  // so that the column-major S is stored with coalesced writes
  auto step = [&](const POp<MX>* aa, const POp<MX>* bb) {
#pragma unroll
    for (int I = 0; I < NI; ++I)
#pragma unroll
      for (int J = 0; J < NJ; ++J) acc[I][J].mac(bb[J], aa[I]);
  };
  constexpr int kRing = 4;
  POp<MX> a[kRing][NI], b[kRing][NJ];
  // drain the previous pass (its stores and unused prefetches), so that the
  // wait counts inside the loop below are exact
  __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
  for (int st = 0; st < kRing - 1; ++st) {
    load(jb + 4 * st + kq, a[st], b[st]);
    __builtin_amdgcn_sched_barrier(0);
  }
  const int nst = (je - jb + 3) / 4;
  int j0 = jb;
  // the scheduling barriers keep every load kRing - 1 steps ahead of its use
  // (the scheduler would otherwise sink the loads to the end of the body)
  for (int n = nst / kRing; n > 0; --n, j0 += 4 * kRing) {
#pragma unroll
    for (int st = 0; st < kRing; ++st) {
      load(j0 + 4 * (st + kRing - 1) + kq, a[(st + kRing - 1) % kRing], b[(st + kRing - 1) % kRing]);
      __builtin_amdgcn_sched_barrier(0);
      step(a[st], b[st]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int st = 0; st < kRing - 1; ++st)
    if (st < nst % kRing) step(a[st], b[st]);
}

// Stacked projection (mixed form), one wave per tile of up to 64 stacked rows
// of blocks sharing W: lane l owns stacked row l, and the 4x4x1 MFMA (16
// blocks of 4 x 4) runs with its A operand broadcast from block c (CBSZ 4,
// ABID c), so that lane 4 c + v supplies W[j][4 c + v] to every block and
// the product lands in lane l, register v as S(row l, column 4 c + v).  One
// load of R and one of W per column j of s feed 4 NC MFMAs; no dimension is
// padded beyond the column groups of 4 and the tile's last rows.
template <int C>
__device__ __forceinline__ void pst_mac(float wr, float wi, float rr, float ri, float nri,
                                        fvec4& re, fvec4& im) {
  re = __builtin_amdgcn_mfma_f32_4x4x1f32(wr, rr, re, 4, C, 0);
  re = __builtin_amdgcn_mfma_f32_4x4x1f32(wi, nri, re, 4, C, 0);
  im = __builtin_amdgcn_mfma_f32_4x4x1f32(wr, ri, im, 4, C, 0);
  im = __builtin_amdgcn_mfma_f32_4x4x1f32(wi, rr, im, 4, C, 0);
}

template <int... C>
__device__ __forceinline__ void pst_macs(std::integer_sequence<int, C...>, float2 w, float2 r,
                                         fvec4* re, fvec4* im) {
  const float nri = -r.y;
  (pst_mac<C>(w.x, w.y, r.x, r.y, nri, re[C], im[C]), ...);
}

template <int NC>
__device__ __forceinline__ void pst_tile(const PTileDev& t, const PBlkDev* blks,
                                         const double* omega) {
  typedef float fv2 __attribute__((ext_vector_type(2)));
  using GP = const __attribute__((address_space(1))) fv2*;
  constexpr int kRing = 12;
  const int lane = threadIdx.x & 63;
  // ranks of the tile's blocks in lanes q < nblk, their first stacked rows
  // (relative to the tile) by an exclusive prefix sum, then this lane's block
  const int ktq = lane < t.nblk ? blks[t.blk0 + lane].kt : 0;
  int incl = ktq;
  for (int o = 1; o < 64; o <<= 1) {
    int v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  const int start = incl - ktq - t.i0;
  const int m = min(lane, t.rows - 1);
  int myq = 0, i = m + t.i0;
  for (int q = 1; q < t.nblk; ++q) {
    int sq = __builtin_amdgcn_readlane(start, q);
    if (m >= sq) {
      myq = q;
      i = m - sq;
    }
  }
  const PBlkDev B = blks[t.blk0 + myq];
  const int kt = B.kt, ns = t.ns, ks = t.ks;
  const GP Rp = (GP)(B.R + i);                    // column j at Rp[j * kt]
  const GP Wp = (GP)(t.W + min(lane, ks - 1));    // row j at Wp[j * ks]
  fvec4 re[NC], im[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) re[c] = im[c] = fvec4{0.0f, 0.0f, 0.0f, 0.0f};
  fv2 rv[kRing], wv[kRing];
  auto load = [&](int j, int st) {
    const int jc = min(j, ns - 1);
    rv[st] = Rp[(int64_t)jc * kt];
    wv[st] = Wp[(int64_t)jc * ks];
  };
  auto mac = [&](int st) {
    pst_macs(std::make_integer_sequence<int, NC>{}, make_float2(wv[st].x, wv[st].y),
             make_float2(rv[st].x, rv[st].y), re, im);
  };
  // columns of s kRing - 1 ahead of their use, in an unrolled ring
#pragma unroll
  for (int st = 0; st < kRing - 1; ++st) {
    load(st, st);
    __builtin_amdgcn_sched_barrier(0);
  }
  int j0 = 0;
  for (int n = ns / kRing; n > 0; --n, j0 += kRing) {
#pragma unroll
    for (int st = 0; st < kRing; ++st) {
      load(j0 + st + kRing - 1, (st + kRing - 1) % kRing);
      __builtin_amdgcn_sched_barrier(0);
      mac(st);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int st = 0; st < kRing - 1; ++st)
    if (st < ns % kRing) mac(st);
  if (lane < t.rows) {
    const double om = omega[B.b];
    float2* Sr = B.S + i;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int col = 4 * c + v;
        if (col < ks) put(Sr, (int64_t)col * kt, make_double2(om * re[c][v], om * im[c][v]));
      }
  }
}

// Every tile of one launch has ceil(ks / 4) = NC column groups (one
// instance per NC: a launch runs one loop body; WPE bounds the registers so
// that WPE or more waves share a SIMD).
template <int NC, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void k_project_stacked(
    const PTileDev* tiles, int64_t ntiles, const PBlkDev* blks, const double* omega) {
  // XCD-aware order, as in k_project_tiled
  unsigned nb = gridDim.x, bx = blockIdx.x;
  unsigned x = bx & 7u, loc = bx >> 3, qx = nb >> 3, rmd = nb & 7u;
  unsigned slot = x * qx + (x < rmd ? x : rmd) + loc;
  int64_t ti = (int64_t)slot * 4 + wave_id();
  if (ti >= ntiles) return;
  static_assert(NC >= 1 && NC <= 16, "column groups");
  pst_tile<NC>(tiles[ti], blks, omega);
}

template <bool MX, int NI, int NJ>
__device__ void proj_store(const ProjDev& t, int ti0, double om, PAcc<MX> (&acc)[NI][NJ]) {
  int lane = threadIdx.x & 63, row = lane & 15;
  using SE = typename std::conditional<MX, float2, double2>::type;
  SE* Sb = static_cast<SE*>(t.S);
#pragma unroll
  for (int I = 0; I < NI; ++I)
#pragma unroll
    for (int J = 0; J < NJ; ++J) {
      int i = 16 * (ti0 + I) + row;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int jj = 16 * J + acc[I][J].row(lane, v);
        double2 z = acc[I][J].get(v);
        if (i < t.kt && jj < t.ks) put(Sb, i + (int64_t)jj * t.kt, make_double2(om * z.x, om * z.y));
      }
    }
}

// Tasks of one launch share (NI, NJ): NJ = column tiles, NI = row tiles per
// pass (the register budget allows at most 16 mixed or 8 FP64 tile pairs).
// SPLIT = 1: one wave per task.  SPLIT = 4 (long column ranges): the four
// waves of a workgroup take a quarter of the columns each and the partial
// sums are added in a fixed order through LDS.
template <bool MX, int NI, int NJ, int SPLIT>
__global__ __launch_bounds__(256) void k_project_tiled(const ProjDev* tasks, int64_t ntasks,
                                                       const double* omega) {
  using AT = typename std::conditional<MX, float, double>::type;
  constexpr int NE = NI * NJ * 4 * 64;  // accumulator elements of one wave
  __shared__ AT red_re[SPLIT > 1 ? 4 * NE : 1], red_im[SPLIT > 1 ? 4 * NE : 1];
  // XCD-aware order: workgroup b runs on XCD b % 8; give each XCD a
  // contiguous range of workgroup slots
  unsigned nb = gridDim.x, b = blockIdx.x;
  unsigned x = b & 7u, loc = b >> 3, q = nb >> 3, rmd = nb & 7u;
  unsigned slot = x * q + (x < rmd ? x : rmd) + loc;
  const int w = wave_id(), lane = threadIdx.x & 63;
  int64_t ti = SPLIT > 1 ? (int64_t)slot : (int64_t)slot * 4 + w;
  if (ti >= ntasks) return;
  const ProjDev t = tasks[ti];
  if (t.kt == 0 || t.ks == 0) return;
  double om = omega[t.b];
  int nti = (t.kt + 15) / 16;
  for (int ti0 = 0; ti0 < nti; ti0 += NI) {
    PAcc<MX> acc[NI][NJ];
    if constexpr (SPLIT == 1) {
      proj_acc<MX, NI, NJ>(t, ti0, 0, t.ns, acc);
      proj_store<MX, NI, NJ>(t, ti0, om, acc);
    } else {
      int part = ((t.ns + 4 * SPLIT - 1) / (4 * SPLIT)) * 4;
      int jb = w * part, je = min(t.ns, jb + part);
      if (jb < je) proj_acc<MX, NI, NJ>(t, ti0, jb, je, acc);
#pragma unroll
      for (int I = 0; I < NI; ++I)
#pragma unroll
        for (int J = 0; J < NJ; ++J)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            int e = ((I * NJ + J) * 4 + v) * 64 + lane;
            red_re[w * NE + e] = acc[I][J].re[v];
            red_im[w * NE + e] = acc[I][J].im[v];
          }
      __syncthreads();
      // the four partial sums in a fixed order, stored by all threads
      for (int e = threadIdx.x; e < NE; e += 256) {
        AT re = red_re[e], im = red_im[e];
#pragma unroll
        for (int src = 1; src < 4; ++src) {
          re += red_re[src * NE + e];
          im += red_im[src * NE + e];
        }
        int pr = e >> 8, v = (e >> 6) & 3, l = e & 63;
        int I = pr / NJ, J = pr - I * NJ;
        int i = 16 * (ti0 + I) + (l & 15);
        int jj = 16 * J + (MX ? f32_row(l, v) : f64_row(l, v));
        if (i < t.kt && jj < t.ks)
          put(static_cast<typename std::conditional<MX, float2, double2>::type*>(t.S),
              i + (int64_t)jj * t.kt, make_double2(om * (double)re, om * (double)im));
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Near field: G|_b column-major per inadmissible block.
// ---------------------------------------------------------------------------
template <int SRC, typename SE>
__global__ __launch_bounds__(256) void k_near(GeomDev g, const int64_t* t_off, const int64_t* t_len,
                                              const int64_t* s_off, const int64_t* s_len,
                                              const int64_t* out_off, SE* out) {
  int64_t b = blockIdx.x;
  int64_t to = t_off[b], tl = t_len[b], so = s_off[b], sl = s_len[b];
  SE* o = out + out_off[b];
  for (int64_t e = threadIdx.x; e < tl * sl; e += 256) {
    int64_t j = e / tl, i = e - j * tl;
    put(o, e, entry<SRC>(g, to + i, so + j, 0));
  }
}

// ---------------------------------------------------------------------------
// Matrix-vector product kernels (verification path, VALU).
// ---------------------------------------------------------------------------
// Work vectors hold nr right-hand sides interleaved: entry p of right-hand
// side q at [p * nr + q] (nr <= NR, a compile-time bound); x and y of the
// caller are column-major, x[q * n + i].  Every kernel reads each element of
// the representation once for all nr right-hand sides.
__global__ void k_gather_perm(const double2* x, const int64_t* perm, int64_t n, int nr,
                              double2* xp) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t src = perm[p];
  for (int q = 0; q < nr; ++q) xp[p * nr + q] = x[(int64_t)q * n + src];
}
__global__ void k_scatter_perm(const double2* yp, const int64_t* perm, int64_t n, int nr,
                               double2* y) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t dst = perm[p];
  for (int q = 0; q < nr; ++q) y[(int64_t)q * n + dst] = yp[p * nr + q];
}

// s[q] += sum_c op(a[c * as]) v[c * nr + q] over c < n for the nr right-hand
// sides (op: conj when conj_a), with U terms loaded ahead of their products
// (U = 4 for one or two right-hand sides, fewer for more) so that several
// loads are in flight.
// Loads and stores through global (address space 1) pointers: a generic
// (flat) access also counts against the LDS wait counter, so that waits for
// LDS operands would also wait for memory traffic in flight.  Native vector
// types carry the address space; the HIP vector types do not.
typedef double gdv2 __attribute__((ext_vector_type(2)));
typedef float gfv2 __attribute__((ext_vector_type(2)));
typedef double gdv4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ double2 ldg(const double2* p, int64_t i) {
  const gdv2 v = ((const __attribute__((address_space(1))) gdv2*)p)[i];
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 ldg(const float2* p, int64_t i) {
  const gfv2 v = ((const __attribute__((address_space(1))) gfv2*)p)[i];
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ double4 ldg(const double4* p, int64_t i) {
  const gdv4 v = ((const __attribute__((address_space(1))) gdv4*)p)[i];
  return make_double4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void stg(double2* p, int64_t i, double2 v) {
  ((__attribute__((address_space(1))) gdv2*)p)[i] = gdv2{v.x, v.y};
}
__device__ __forceinline__ void stg(float2* p, int64_t i, float2 v) {
  ((__attribute__((address_space(1))) gfv2*)p)[i] = gfv2{v.x, v.y};
}

// s[q] += sum_{c < n} op(a[c as]) v[c vs + q] (q < nr; vs = nr unless given),
// op the conjugate when conj_a; U terms loaded ahead of their products
template <int NR, typename AE = double2>
__device__ __forceinline__ void dot_rhs(double2 (&s)[NR], const AE* a, int64_t as,
                                        const double2* v, int64_t n, int nr, bool conj_a,
                                        int64_t vs = 0) {
  constexpr int U = NR == 1 ? 8 : (NR == 2 ? 4 : (NR <= 4 ? 2 : 1));
  const int64_t vst = vs ? vs : nr;
  int64_t c = 0;
  for (; c + U <= n; c += U) {
    double2 av[U], xv[U][NR];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      av[u] = wide(ldg(a, (c + u) * as));
#pragma unroll
      for (int q = 0; q < NR; ++q)
        if (q < nr) xv[u][q] = ldg(v, (c + u) * vst + q);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < NR; ++q)
        if (q < nr) {
          double2 t = conj_a ? cmulc(av[u], xv[u][q]) : cmul(av[u], xv[u][q]);
          s[q].x += t.x;
          s[q].y += t.y;
        }
  }
  for (; c < n; ++c) {
    const double2 ac = wide(ldg(a, c * as));
#pragma unroll
    for (int q = 0; q < NR; ++q)
      if (q < nr) {
        const double2 xq = ldg(v, c * vst + q);
        double2 t = conj_a ? cmulc(ac, xq) : cmul(ac, xq);
        s[q].x += t.x;
        s[q].y += t.y;
      }
  }
}

// s += sum_{c < m} op(a[c as]) xs[c] for the lane's row, the vector entries
// in LDS (the same entry for every lane of a slot: a broadcast read), U
// terms of a loaded ahead of their products
template <typename AE>
__device__ __forceinline__ void dot_lds(double2& s, const AE* a, int64_t as, const double2* xs,
                                        int m, bool conj_a) {
  constexpr int U = 8;
  int c = 0;
  for (; c + U <= m; c += U) {
    double2 av[U];
#pragma unroll
    for (int u = 0; u < U; ++u) av[u] = wide(ldg(a, (int64_t)(c + u) * as));
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double2 xq = xs[c + u];
      const double2 t = conj_a ? cmulc(av[u], xq) : cmul(av[u], xq);
      s.x += t.x;
      s.y += t.y;
    }
  }
  for (; c < m; ++c) {
    const double2 ac = wide(ldg(a, (int64_t)c * as));
    const double2 xq = xs[c];
    const double2 t = conj_a ? cmulc(ac, xq) : cmul(ac, xq);
    s.x += t.x;
    s.y += t.y;
  }
}

// forward, leaf items: xh = Q^* x|t
template <int NR>
__global__ __launch_bounds__(128) void k_fwd_leaf(const ItemDev* items, const int32_t* litems,
                                                  const int64_t* xh_off, const double2* xp,
                                                  double2* xh, int nr) {
  int32_t i = litems[blockIdx.x];
  const ItemDev& it = items[i];
  int k = it.k;
  for (int kk = threadIdx.x; kk < k; kk += blockDim.x) {
    double2 s[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) s[q] = make_double2(0.0, 0.0);
    dot_rhs<NR>(s, it.Q + kk, k, xp + it.row_off * nr, it.m, nr, true);
#pragma unroll
    for (int q = 0; q < NR; ++q)
      if (q < nr) xh[(xh_off[i] + kk) * nr + q] = s[q];
  }
}

// forward, non-leaf items: xh_tc = Q_hat^* [xh_t1c'; xh_t2c']
template <int NR>
__global__ __launch_bounds__(128) void k_fwd_inner(const ItemDev* items, const int32_t* litems,
                                                   const int64_t* xh_off, double2* xh, int nr) {
  int32_t i = litems[blockIdx.x];
  const ItemDev& it = items[i];
  int k = it.k;
  const ItemDev& s1 = items[it.son[0]];
  const int64_t o1 = xh_off[it.son[0]], o2 = xh_off[it.son[1]] - s1.k;
  for (int kk = threadIdx.x; kk < k; kk += blockDim.x) {
    double2 s[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) s[q] = make_double2(0.0, 0.0);
    dot_rhs<NR>(s, it.Q + kk, k, xh + o1 * nr, s1.k, nr, true);
    dot_rhs<NR>(s, it.Q + (int64_t)s1.k * k + kk, k, xh + (o2 + s1.k) * nr, it.r - s1.k, nr,
                true);
#pragma unroll
    for (int q = 0; q < NR; ++q)
      if (q < nr) xh[(xh_off[i] + kk) * nr + q] = s[q];
  }
}

// coupling: yh_i = sum over the item's blocks of S_b xh_partner (or S_b^* for
// the adjoint, where S_b is kr x kc with the item on the column side).  The
// matrices come oriented with the item's coefficients as rows: S_b for op
// N, the transposed copy S_b^T (kc x kr, column-major) for the adjoint, so
// that both read consecutive rows across the lanes.  Items are taken in the
// order given (most work first): the first nheavy workgroups take one item
// each with their four waves, the others four items, one per wave.  Each
// wave is cut into 64 / kp slots of kp lanes (kp the power of two >= k, at
// least 8), lane kk of a slot one coefficient; the slots of the item's waves
// take its blocks in turn, and their sums are added with shuffles, then
// across the waves through LDS, in a fixed order.  The partner's
// coefficients are the same for all lanes of a slot.
template <int NR, typename SE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NR == 1 ? 5 : 1))) void k_coupling(const ItemDev* items, int32_t nitems,
                                                  int32_t nheavy, const int32_t* order,
                                                  const int64_t* cbegin, const int32_t* cblock,
                                                  const int32_t* cpartner,
                                                  const void* const* S_ptr,
                                                  const int32_t* S_rows, const int32_t* S_cols,
                                                  const int64_t* xh_off, const double2* xh,
                                                  const int64_t* yh_off, double2* yh,
                                                  int adjoint, int nr) {
  __shared__ double2 part[4][NR][64];
  // one right-hand side: the partner's coefficients of the current block,
  // kp per slot, staged in LDS instead of loaded by every lane per column
  __shared__ double2 xsh[NR == 1 ? 4 * 64 : 1];
  const int w = wave_id();
  const bool heavy = (int32_t)blockIdx.x < nheavy;  // the same for the whole workgroup
  const int32_t wi = heavy ? (int32_t)blockIdx.x
                           : nheavy + ((int32_t)blockIdx.x - nheavy) * 4 + w;
  if (wi >= nitems) return;  // light workgroups only: heavy ones have an item
  const int32_t i = order[wi];
  const int lane = threadIdx.x & 63;
  const int k = items[i].k;
  const int kp = k <= 8 ? 8 : (k <= 16 ? 16 : (k <= 32 ? 32 : 64));
  const int nslot = 64 / kp, sl = lane / kp, kl = lane % kp;
  const int first = (heavy ? w * nslot : 0) + sl, stride = (heavy ? 4 : 1) * nslot;
  for (int kk0 = 0; kk0 < k; kk0 += 64) {
    const int kk = min(kk0 + kl, k - 1);
    double2 s[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) s[q] = make_double2(0.0, 0.0);
    for (int64_t c = cbegin[i] + first; c < cbegin[i + 1]; c += stride) {
      const int32_t b = cblock[c];
      const SE* Sb = static_cast<const SE*>(S_ptr[b]);
      const int kr = S_rows[b], kc = S_cols[b];  // of the oriented matrix
      const double2* x = xh + xh_off[cpartner[c]] * nr;
      // op N: sum_jj S[kk, jj] x[jj]; adjoint: sum_jj conj(S^T[kk, jj]) x[jj]
      if constexpr (NR == 1) {
        double2* xs = xsh + 64 * w + sl * kp;
        for (int j0 = 0; j0 < kc; j0 += kp) {
          const int m = min(kp, kc - j0);
          wave_sync();  // the slot's reads of the previous entries are done
          if (kl < m) xs[kl] = ldg(x, j0 + kl);
          wave_sync();
          dot_lds(s[0], Sb + kk + (int64_t)j0 * kr, kr, xs, m, adjoint != 0);
        }
      } else {
        dot_rhs<NR>(s, Sb + kk, kr, x, kc, nr, adjoint != 0);
      }
    }
    for (int o = kp; o < 64; o <<= 1)
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        s[q].x += __shfl_xor(s[q].x, o, 64);
        s[q].y += __shfl_xor(s[q].y, o, 64);
      }
    if (heavy) {
#pragma unroll
      for (int q = 0; q < NR; ++q) part[w][q][lane] = s[q];
      __syncthreads();
      if (w == 0) {
#pragma unroll
        for (int q = 0; q < NR; ++q)
#pragma unroll
          for (int u = 1; u < 4; ++u) {
            s[q].x += part[u][q][lane].x;
            s[q].y += part[u][q][lane].y;
          }
      }
      __syncthreads();
    }
    if ((!heavy || w == 0) && sl == 0 && kk0 + kl < k)
#pragma unroll
      for (int q = 0; q < NR; ++q)
        if (q < nr) yh[(yh_off[i] + kk0 + kl) * nr + q] = s[q];
  }
}

// backward to the sons: yh_{t'c'} += sum over father items (fa,c+) with
// sd(c+) = c' of E_{t'c+} yh_{fa c+}; E_{t'c+} = rows of the father's factor.
template <int NR>
__global__ __launch_bounds__(128) void k_bwd_inner(const ItemDev* items, const int32_t* litems,
                                                   const int64_t* fbegin, const int32_t* fitem,
                                                   const int32_t* fsonidx, const int64_t* yh_off,
                                                   double2* yh, int nr) {
  int32_t i = litems[blockIdx.x];
  const ItemDev& it = items[i];
  int k = it.k;
  for (int kk = threadIdx.x; kk < k; kk += blockDim.x) {
    double2 s[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) s[q] = q < nr ? yh[(yh_off[i] + kk) * nr + q] : make_double2(0, 0);
    for (int64_t c = fbegin[blockIdx.x]; c < fbegin[blockIdx.x + 1]; ++c) {
      const ItemDev& fa = items[fitem[c]];
      int rowoff = fsonidx[c] == 0 ? 0 : items[fa.son[0]].k;
      const double2* y = yh + yh_off[fitem[c]] * nr;
      dot_rhs<NR>(s, fa.Q + (int64_t)(rowoff + kk) * fa.k, 1, y, fa.k, nr, false);
    }
#pragma unroll
    for (int q = 0; q < NR; ++q)
      if (q < nr) yh[(yh_off[i] + kk) * nr + q] = s[q];
  }
}

// leaf rows: y|L = sum_c Q_Lc yh_Lc + near-field rows of L.  One workgroup
// of four waves per task (the basis terms of a leaf, added to the rows
// already written (accumulate), or a leaf's near-field blocks, or a part of them),
// lane j one row of the leaf (leaves have at most 64 rows): the waves take
// the task's basis terms in turn, or the columns of each near-field block in
// turn (the workgroup streams one block at a time), and the partial sums
// are added through LDS in wave order.  The adjoint reads the transposed
// copy of every near-field block (nearT, #s x #t column-major), so that both
// products read consecutive rows across the lanes.  The two kinds of task
// are separate instantiations (NEAR), so that each keeps only the registers
// of its own loop (with eight right-hand sides both run at five waves per
// SIMD, against two for one kernel holding both loops).
template <int NR, bool NEAR, typename SE>
__global__ __launch_bounds__(256) void k_bwd_leaf(const ItemDev* items, const LeafDev* leaves,
                                                  const NearRefDev* nref, const NearDev* nears,
                                                  const void* nearv, const void* nearT,
                                                  const int64_t* yh_off, const double2* yh,
                                                  const double2* xp, double2* yp,
                                                  double2* partial, int adjoint, int nr,
                                                  int accumulate) {
  __shared__ double2 part[4][NR][64];
  const LeafDev L = leaves[blockIdx.x];
  const int w = wave_id(), lane = threadIdx.x & 63;
  const int j = min(lane, L.len - 1);
  double2 s[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) s[q] = make_double2(0.0, 0.0);
  if constexpr (!NEAR) {
    for (int q = L.item_first + w; q < L.item_first + L.item_count; q += 4) {
      const ItemDev& it = items[q];
      dot_rhs<NR>(s, it.Q + (int64_t)j * it.k, 1, yh + yh_off[q] * nr, it.k, nr, false);
    }
  }
  if constexpr (NEAR) for (int64_t q = L.near_begin; q < L.near_end; ++q) {
    const NearRefDev ref = nref[q];
    const NearDev nb = nears[ref.b];
    const int64_t row = ref.row0 + j;
    // op N: sum_c B[row, c] x[s_off + c]; adjoint: sum_c conj(B^T[row, c])
    // x[t_off + c] with B^T the transposed copy (#s x #t); row = ref.row0 + j.
    // The four waves take the block's columns in turn (one stream per
    // workgroup).
    const int64_t ld = adjoint ? nb.s_len : nb.t_len;
    const int64_t ncol = adjoint ? nb.t_len : nb.s_len;
    const int64_t xo = adjoint ? nb.t_off : nb.s_off;
    const SE* B = static_cast<const SE*>(adjoint ? nearT : nearv) + nb.off + row;
    if (w < ncol)
      dot_rhs<NR>(s, B + w * ld, 4 * ld, xp + (xo + w) * nr, (ncol - w + 3) / 4, nr, adjoint != 0,
                  4 * (int64_t)nr);
  }
#pragma unroll
  for (int q = 0; q < NR; ++q) part[w][q][lane] = s[q];
  __syncthreads();
  if (w == 0 && lane < L.len) {
    double2* out = L.slot < 0 ? yp + (L.row_off + lane) * nr
                              : partial + ((int64_t)L.slot * 64 + lane) * nr;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      if (q < nr) {
        double2 t = part[0][q][lane];
#pragma unroll
        for (int u = 1; u < 4; ++u) {
          t.x += part[u][q][lane].x;
          t.y += part[u][q][lane].y;
        }
        if (accumulate) {
          const double2 o = out[q];
          t.x += o.x;
          t.y += o.y;
        }
        out[q] = t;
      }
    }
  }
}

// rows of the leaves whose work was split: the partial sums of their slots
// added in slot order (one wave per leaf)
template <int NR>
__global__ __launch_bounds__(64) void k_leaf_sum(const LeafDev* leaves, const double2* partial,
                                                 double2* yp, int nr) {
  const LeafDev L = leaves[blockIdx.x];
  const int lane = threadIdx.x;
  if (lane >= L.len) return;
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    if (q < nr) {
      double2 t = make_double2(0.0, 0.0);
      for (int sl = L.item_first; sl < L.item_first + L.item_count; ++sl) {
        const double2 v = partial[((int64_t)sl * 64 + lane) * nr + q];
        t.x += v.x;
        t.y += v.y;
      }
      yp[(L.row_off + lane) * nr + q] = t;
    }
  }
}

// transposed copy of the near-field blocks for the adjoint (one workgroup
// per block, tiles of 64 rows x 32 columns through LDS)
template <typename SE>
__global__ __launch_bounds__(256) void k_near_transpose(const NearDev* nears, const SE* B,
                                                        SE* BT) {
  __shared__ SE tile[32][65];
  const NearDev nb = nears[blockIdx.x];
  const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;  // loads: 64 rows x 4
  const int sx = threadIdx.x & 31, sy = threadIdx.x >> 5;  // stores: 32 columns x 8
  for (int64_t i0 = 0; i0 < nb.t_len; i0 += 64)
    for (int64_t j0 = 0; j0 < nb.s_len; j0 += 32) {
      for (int jj = ly; jj < 32; jj += 4) {
        const int64_t i = i0 + lx, j = j0 + jj;
        if (i < nb.t_len && j < nb.s_len) tile[jj][lx] = B[nb.off + i + j * nb.t_len];
      }
      __syncthreads();
      for (int ii = sy; ii < 64; ii += 8) {
        const int64_t j = j0 + sx, i = i0 + ii;
        if (i < nb.t_len && j < nb.s_len) BT[nb.off + j + i * nb.s_len] = tile[sx][ii];
      }
      __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Direct products with the matrix (FP64): y_i = sum_j G_ij x_j (op 'N') or
// y_i = sum_j conj(G_ji) x_j (op 'C'); rows are permuted positions.
// ---------------------------------------------------------------------------
template <int SRC>
__global__ __launch_bounds__(256) void k_direct(GeomDev g, const int64_t* rows, int64_t nrows,
                                                const double2* xp, int adjoint, double2* out) {
  __shared__ double2 red[256];
  int64_t q = blockIdx.x;
  if (q >= nrows) return;
  int64_t i = rows ? rows[q] : q;
  double2 s = make_double2(0.0, 0.0);
  for (int64_t j = threadIdx.x; j < g.n; j += 256) {
    double2 e = adjoint ? entry<SRC>(g, i, j, 1) : entry<SRC>(g, i, j, 0);
    double2 v = cmul(e, xp[j]);
    s.x += v.x;
    s.y += v.y;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red[threadIdx.x].x += red[threadIdx.x + o].x;
      red[threadIdx.x].y += red[threadIdx.x + o].y;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[q] = red[0];
}

// ---------------------------------------------------------------------------
// Wave-level pipelines.  Each wave owns a work unit and builds exactly the
// MFMA operands it consumes: no block barriers.  MX selects the mixed form:
// entries with FP32 polynomials, R stored in complex FP32, R-products on
// FP32 MFMA; Gram matrices are accumulated in FP64 in both forms.
// ---------------------------------------------------------------------------

// Column data of the leaf block rows of one level, written once per level:
// one workgroup per item walks its column-set entries.  Column j of the
// weighted block row carries (x, y, z, factor): Helmholtz factor =
// scale * (side 0 ? w_j : 1) / (4 pi), scale = 1 / (omega_b zeta^d); dense:
// the original index in x and factor = scale.  Double layer, mixed form
// (pos_dlp): (x, y, z, factor) as for the single layer, followed after the
// item's N columns by the unit normals (nx, ny, nz, 0); FP64 form: the
// position in x and factor = scale.
template <int SRC>
__global__ __launch_bounds__(256) void k_leaf_cols(GeomDev g, const ItemDev* items,
                                                   const int32_t* litems, const EntDev* ents,
                                                   int side, int pos_dlp) {
  const ItemDev& it = items[litems[blockIdx.x]];
  double4* out = it.cols;
  // the four waves take the column-set entries in turn, so that the loads
  // of several entries are in flight at once
  const int lane = threadIdx.x & 63;
  for (int64_t e = it.ent_begin + wave_id(); e < it.ent_end; e += 4) {
    const EntDev en = ents[e];
    for (int64_t q = lane; q < en.len; q += 64) {
      int64_t pos = en.pos + q;
      double4 v;
      if (SRC == SRC_HELMHOLTZ || (SRC == SRC_DLP && pos_dlp)) {
        const double* p = g.pts + 4 * pos;
        v = make_double4(p[0], p[1], p[2], en.scale * (side == 0 ? p[3] : 1.0) * kInv4Pi);
        if (SRC == SRC_DLP) {
          const double* nv = g.nrm + 4 * pos;
          out[it.N + en.col_start + q] = make_double4(nv[0], nv[1], nv[2], 0.0);
        }
      } else {
        // dense: original index; double layer: position
        const int64_t id = SRC == SRC_DLP ? pos : g.perm[pos];
        v = make_double4(__longlong_as_double((long long)id), 0.0, 0.0, en.scale);
      }
      out[en.col_start + q] = v;
    }
  }
}

struct RowData {
  double x, y, z, f;   // Helmholtz: coordinates and row factor; dense: original index in x
};

// Padding rows and columns of the Helmholtz block rows: factor 0 at points far
// from every real point and from each other, so that their entries are 0
// without a distance clamp.
constexpr double kPadRow = 1.0e10;
__device__ __forceinline__ double4 pad_col() { return make_double4(-1.0e10, 0.0, 0.0, 0.0); }

// far: padding rows of the mixed-form generator sit at kPadRow (the FP64
// generator clamps the distance and keeps them at the origin)
template <int SRC>
__device__ __forceinline__ RowData row_data(const GeomDev& g, const ItemDev& it, int rho, int side,
                                            bool far = false) {
  RowData r{SRC == SRC_HELMHOLTZ && far ? kPadRow : 0.0, 0.0, 0.0, 0.0};
  if (rho < it.m) {
    int64_t pos = it.row_off + rho;
    if constexpr (SRC == SRC_HELMHOLTZ) {
      const double* p = g.pts + 4 * pos;
      r.x = p[0];
      r.y = p[1];
      r.z = p[2];
      r.f = side == 1 ? p[3] : 1.0;
    } else {
      r.x = __longlong_as_double((long long)(SRC == SRC_DLP ? pos : g.perm[pos]));
      r.f = 1.0;
    }
  }
  return r;
}

// unit normal of row rho (double layer; 0 for padding rows)
__device__ __forceinline__ double4 row_normal(const GeomDev& g, const ItemDev& it, int rho) {
  double4 n = make_double4(0.0, 0.0, 0.0, 0.0);
  if (rho < it.m) {
    const double* v = g.nrm + 4 * (it.row_off + rho);
    n = make_double4(v[0], v[1], v[2], 0.0);
  }
  return n;
}

// Entry of the weighted block row from staged row and column data.  No
// branch: padding rows and columns carry factor 0 (the distance is clamped so
// that 0 * 1/r stays 0), which lets the compiler interleave several entries.
template <int SRC, bool MX>
__device__ __forceinline__ double2 gen_entry(const GeomDev& g, const RowData& rw, double4 cc,
                                             int side) {
  double f = rw.f * cc.w;
  if constexpr (SRC == SRC_HELMHOLTZ) {
    double dx = rw.x - cc.x, dy = rw.y - cc.y, dz = rw.z - cc.z;
    double r2 = fmax(dx * dx + dy * dy + dz * dz, 1e-300);
    double ri = rsqrt_nr(r2);
    if constexpr (MX) {
      float sn, cs;
      sincos_mixed(g.kappa * (r2 * ri), sn, cs);
      float a = (float)(f * ri);
      return make_double2(a * cs, side == 0 ? a * sn : -a * sn);
    } else {
      double sn, cs;
      sincos_phase(g.kappa * (r2 * ri), sn, cs);
      double a = f * ri;
      return make_double2(a * cs, side == 0 ? a * sn : -a * sn);
    }
  } else if constexpr (SRC == SRC_DLP) {
    int64_t i = (int64_t)__double_as_longlong(rw.x), j = (int64_t)__double_as_longlong(cc.x);
    double2 v = dlp_entry(g, i, j, side);
    return make_double2(v.x * f, v.y * f);
  } else {
    const double2* G = reinterpret_cast<const double2*>(g.G);
    int64_t i = (int64_t)__double_as_longlong(rw.x), j = (int64_t)__double_as_longlong(cc.x);
    double2 v = side == 0 ? G[i * g.ldg + j] : G[j * g.ldg + i];
    return make_double2(v.x * f, (side == 0 ? v.y : -v.y) * f);
  }
}

// Mixed form, Helmholtz: the same entry as complex FP32.  The distance and
// the phase are formed in FP64, sin and cos and the amplitude in FP32.
// Padding rows and columns sit far apart (see kPadRow, kPadCol) with factor
// 0, so the entry needs no clamp.
__device__ __forceinline__ float2 gen_entry_mx(const GeomDev& g, const RowData& rw, double4 cc,
                                               int side) {
  double dx = rw.x - cc.x, dy = rw.y - cc.y, dz = rw.z - cc.z;
  double r2 = dx * dx + dy * dy + dz * dz;
  // 1/r: the hardware estimate (about 2^-24 relative) refined by one Newton
  // step; r = r2 / r to full FP64 accuracy
  double r0 = __builtin_amdgcn_rsq(r2);
  double e = fma(-r2 * r0, r0, 1.0);
  double ri = fma(0.5 * r0, e, r0);
  float sn, cs;
  sincos_mixed(g.kappa * (r2 * ri), sn, cs);
  float a = (float)rw.f * (float)cc.w * (float)ri;
  return make_float2(a * cs, side == 0 ? a * sn : -a * sn);
}

// Mixed form, double layer: w_q (1 - i kappa r) exp(i kappa r) <x_p - x_q,
// n_q> / (4 pi r^3) with q the column point (side 0) or the row point (side
// 1, conjugated); the distance, <x_p - x_q, n_q> and the phase reduction in
// FP64, sin, cos and the amplitude in FP32.  rn, cn: the row's and the
// column's unit normals.  Padding rows and columns have factor and normal 0
// and sit far apart, so the entry is 0 without a clamp.
__device__ __forceinline__ float2 gen_entry_dlp_mx(const GeomDev& g, const RowData& rw,
                                                   double4 rn, double4 cc, double4 cn,
                                                   int side) {
  double dx = rw.x - cc.x, dy = rw.y - cc.y, dz = rw.z - cc.z;
  double r2 = dx * dx + dy * dy + dz * dz;
  double r0 = __builtin_amdgcn_rsq(r2);
  double e = fma(-r2 * r0, r0, 1.0);
  double ri = fma(0.5 * r0, e, r0);
  double kr = g.kappa * (r2 * ri);
  // <x_p - x_q, n_q>: side 0 (row point p, column point q) or side 1 (row q)
  double dot = side == 0 ? dx * cn.x + dy * cn.y + dz * cn.z
                         : -(dx * rn.x + dy * rn.y + dz * rn.z);
  float sn, cs;
  sincos_mixed(kr, sn, cs);
  float a = (float)(rw.f * cc.w * dot * (ri * ri * ri));
  float k = (float)kr;
  float re = a * fmaf(k, sn, cs), im = a * fmaf(-k, cs, sn);
  return make_float2(re, side == 0 ? im : -im);
}

// Gram of a leaf block row, one unit per wave, all lower tile pairs.  The
// entries of k-step s+1 are generated while the MFMAs of k-step s issue; the
// scheduling hints interleave one MFMA with a group of VALU instructions.
template <int SRC, bool MX, int NT>
__device__ void gram_leaf_wave(const GeomDev& g, const ItemDev& it, const EntDev* ents, int side,
                               const UnitDev& u, double2* out, double4* cl) {
  constexpr int NP = NT * (NT + 1) / 2;
  int lane = threadIdx.x & 63, row = lane & 15, kq = lane >> 4;
  RowData rw[NT];
#pragma unroll
  for (int I = 0; I < NT; ++I) rw[I] = row_data<SRC>(g, it, 16 * I + row, side);
  dvec4 acr[NP], aci[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    acr[p] = dvec4{0, 0, 0, 0};
    aci[p] = dvec4{0, 0, 0, 0};
  }
  double4 cnext = lane < u.ncols ? it.cols[u.col_begin + lane] : make_double4(0.0, 0.0, 0.0, 0.0);
  for (int64_t c0 = 0; c0 < u.ncols; c0 += 64) {
    int64_t left = u.ncols - c0;
    wave_sync();
    cl[lane] = cnext;
    wave_sync();
    // prefetch the next chunk's column data
    cnext = c0 + 64 + lane < u.ncols ? it.cols[u.col_begin + c0 + 64 + lane]
                                     : make_double4(0.0, 0.0, 0.0, 0.0);
    int nks = left >= 64 ? 16 : (int)((left + 3) / 4);
    double2 cur[NT];
    {
      double4 cc = cl[kq];
#pragma unroll
      for (int I = 0; I < NT; ++I) cur[I] = gen_entry<SRC, MX>(g, rw[I], cc, side);
    }
    for (int ks = 0; ks < nks; ++ks) {
      double2 nxt[NT];
      double4 cn = cl[(4 * (ks + 1) + kq) & 63];
      bool more = ks + 1 < nks;
#pragma unroll
      for (int I = 0; I < NT; ++I)
        nxt[I] = more ? gen_entry<SRC, MX>(g, rw[I], cn, side) : make_double2(0.0, 0.0);
      int p = 0;
#pragma unroll
      for (int I = 0; I < NT; ++I) {
#pragma unroll
        for (int J = 0; J <= I; ++J) {
          acr[p] = mfma_f64(cur[I].x, cur[J].x, acr[p]);
          acr[p] = mfma_f64(cur[I].y, cur[J].y, acr[p]);
          aci[p] = mfma_f64(cur[I].y, cur[J].x, aci[p]);
          aci[p] = mfma_f64(-cur[I].x, cur[J].y, aci[p]);
          ++p;
        }
      }
#pragma unroll
      for (int q = 0; q < 4 * NP; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x002, 6, 0);
      }
#pragma unroll
      for (int I = 0; I < NT; ++I) cur[I] = nxt[I];
    }
  }
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int v = 0; v < 4; ++v) out[(p * 4 + v) * 64 + lane] = make_double2(acr[p][v], aci[p][v]);
}

template <int SRC, bool MX>
__global__ __launch_bounds__(256) void k_gram_leaf_w(GeomDev g, const ItemDev* items,
                                                     const EntDev* ents, const UnitDev* units,
                                                     int64_t nunits, int side, double2* partial) {
  __shared__ double4 cls[4][64];
  int w = wave_id();
  int64_t ui = (int64_t)blockIdx.x * 4 + w;
  if (ui >= nunits) return;
  const UnitDev u = units[ui];
  const ItemDev& it = items[u.item];
  int nt = (it.r + 15) / 16;
  double2* out = partial + u.slot_off;
  switch (nt) {
    case 1: gram_leaf_wave<SRC, MX, 1>(g, it, ents, side, u, out, cls[w]); break;
    case 2: gram_leaf_wave<SRC, MX, 2>(g, it, ents, side, u, out, cls[w]); break;
    case 3: gram_leaf_wave<SRC, MX, 3>(g, it, ents, side, u, out, cls[w]); break;
    default: gram_leaf_wave<SRC, MX, 4>(g, it, ents, side, u, out, cls[w]); break;
  }
}

// Row rho of G_hat_tc = zeta [R_t1c' ; R_t2c'] at column j (0 outside).
// Gram of a non-leaf block row, one unit (column range x tile block) per wave.
// Each lane's row of every tile comes from one son, so its source pointer
// and stride are fixed for the unit; loads are unconditional (rows past r
// read row r - 1 and only feed Gram rows and columns that are not kept;
// columns past the unit are clamped and masked to zero at use), four columns
// per k-step, two k-steps ahead in an unrolled ring of three register sets.
// zeta^2 is applied to the finished tiles.
template <bool MX, int NA, int NB, bool DIAG>
__device__ void gram_inner_wave(const ItemDev& it, const ItemDev& s1, const ItemDev& s2,
                                const UnitDev& u, double zeta, double2* out) {
  constexpr int NP = DIAG ? NA * (NA + 1) / 2 : NA * NB;
  constexpr int NL = DIAG ? 0 : NB;
  constexpr int NT = NA + NL;
  using Sc = typename std::conditional<MX, float, double>::type;
  typedef Sc E2 __attribute__((ext_vector_type(2)));
  using GP = const __attribute__((address_space(1))) E2*;
  using OT = typename std::conditional<MX, float2, double2>::type;
  int lane = threadIdx.x & 63, row = lane & 15, kq = lane >> 4;
  const int r = it.r, k1 = s1.k;
  const int ncols = (int)u.ncols;
  const int64_t c0 = it.col_off + u.col_begin;
  GP src[NT];
  int ld[NT];
#pragma unroll
  for (int T = 0; T < NT; ++T) {
    int rho = 16 * (T < NA ? u.a0 + T : u.b0 + (T - NA)) + row;
    int rc = min(rho, r - 1);
    if (rc < k1) {
      src[T] = (GP)(reinterpret_cast<const OT*>(s1.R) + c0 * k1 + rc);
      ld[T] = k1;
    } else {
      src[T] = (GP)(reinterpret_cast<const OT*>(s2.R) + c0 * s2.k + (rc - k1));
      ld[T] = s2.k;
    }
  }
  dvec4 acr[NP], aci[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    acr[p] = dvec4{0, 0, 0, 0};
    aci[p] = dvec4{0, 0, 0, 0};
  }
  auto load = [&](int c, E2* v) {
    const int cc = min(c, ncols - 1);
#pragma unroll
    for (int T = 0; T < NT; ++T) v[T] = src[T][(int64_t)cc * ld[T]];
  };
  auto step = [&](int c, const E2* v) {
    const bool ok = c < ncols;
    double2 x[NT];
#pragma unroll
    for (int T = 0; T < NT; ++T) x[T] = ok ? make_double2(v[T].x, v[T].y) : make_double2(0.0, 0.0);
    int p = 0;
#pragma unroll
    for (int I = 0; I < NA; ++I) {
#pragma unroll
      for (int J = 0; J < (DIAG ? I + 1 : NB); ++J) {
        double2 xa = x[I];
        double2 yb = DIAG ? x[J] : x[NA + J];
        acr[p] = mfma_f64(xa.x, yb.x, acr[p]);
        acr[p] = mfma_f64(xa.y, yb.y, acr[p]);
        aci[p] = mfma_f64(xa.y, yb.x, aci[p]);
        aci[p] = mfma_f64(-xa.x, yb.y, aci[p]);
        ++p;
      }
    }
  };
  E2 v0[NT], v1[NT], v2[NT];
  load(kq, v0);
  __builtin_amdgcn_sched_barrier(0);
  load(4 + kq, v1);
  __builtin_amdgcn_sched_barrier(0);
  const int nst = (ncols + 3) / 4;
  int c = kq;
  for (int n = nst / 3; n > 0; --n, c += 12) {
    load(c + 8, v2);
    __builtin_amdgcn_sched_barrier(0);
    step(c, v0);
    __builtin_amdgcn_sched_barrier(0);
    load(c + 12, v0);
    __builtin_amdgcn_sched_barrier(0);
    step(c + 4, v1);
    __builtin_amdgcn_sched_barrier(0);
    load(c + 16, v1);
    __builtin_amdgcn_sched_barrier(0);
    step(c + 8, v2);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (nst % 3 >= 1) step(c, v0);
  if (nst % 3 == 2) step(c + 4, v1);
  const double z2 = zeta * zeta;
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      out[(p * 4 + v) * 64 + lane] = make_double2(acr[p][v] * z2, aci[p][v] * z2);
}

template <bool MX>
__global__ __launch_bounds__(256) void k_gram_inner_w(const ItemDev* items, const UnitDev* units,
                                                      int64_t nunits, double zeta,
                                                      double2* partial) {
  int w = wave_id();
  int64_t ui = (int64_t)blockIdx.x * 4 + w;
  if (ui >= nunits) return;
  const UnitDev u = units[ui];
  const ItemDev& it = items[u.item];
  const ItemDev& s1 = items[it.son[0]];
  const ItemDev& s2 = items[it.son[1]];
  double2* out = partial + u.slot_off;
  if (u.a0 == u.b0) {
    switch (u.na) {
      case 1: gram_inner_wave<MX, 1, 1, true>(it, s1, s2, u, zeta, out); break;
      case 2: gram_inner_wave<MX, 2, 2, true>(it, s1, s2, u, zeta, out); break;
      case 3: gram_inner_wave<MX, 3, 3, true>(it, s1, s2, u, zeta, out); break;
      default: gram_inner_wave<MX, 4, 4, true>(it, s1, s2, u, zeta, out); break;
    }
  } else {
    if (u.na == 1) {
      switch (u.nb) {
        case 1: gram_inner_wave<MX, 1, 1, false>(it, s1, s2, u, zeta, out); break;
        case 2: gram_inner_wave<MX, 1, 2, false>(it, s1, s2, u, zeta, out); break;
        case 3: gram_inner_wave<MX, 1, 3, false>(it, s1, s2, u, zeta, out); break;
        default: gram_inner_wave<MX, 1, 4, false>(it, s1, s2, u, zeta, out); break;
      }
    } else {
      switch (u.nb) {
        case 1: gram_inner_wave<MX, 2, 1, false>(it, s1, s2, u, zeta, out); break;
        case 2: gram_inner_wave<MX, 2, 2, false>(it, s1, s2, u, zeta, out); break;
        case 3: gram_inner_wave<MX, 2, 3, false>(it, s1, s2, u, zeta, out); break;
        default: gram_inner_wave<MX, 2, 4, false>(it, s1, s2, u, zeta, out); break;
      }
    }
  }
}

// One complex multiply-accumulate of the R-product on MFMA:
// acc += A^T conj(Q) (re = ar qr + ai qi, im = ai qr - ar qi).  Operands are
// complex FP64, or complex FP32 in the mixed form.
template <bool MX>
using ROp = typename std::conditional<MX, float2, double2>::type;

template <bool MX>
__device__ __forceinline__ ROp<MX> rop(double2 v) {
  if constexpr (MX)
    return make_float2((float)v.x, (float)v.y);
  else
    return v;
}

template <bool MX>
struct RAcc;
template <>
struct RAcc<false> {
  dvec4 re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
  __device__ __forceinline__ void mac(double2 a, double2 q) {
    re = mfma_f64(a.x, q.x, re);
    re = mfma_f64(a.y, q.y, re);
    im = mfma_f64(a.y, q.x, im);
    im = mfma_f64(-a.x, q.y, im);
  }
  __device__ __forceinline__ int row(int lane, int v) const { return f64_row(lane, v); }
  __device__ __forceinline__ void store(void* R, int64_t idx, int v, double sc = 1.0) const {
    stg(reinterpret_cast<double2*>(R), idx, make_double2(re[v] * sc, im[v] * sc));
  }
};
template <>
struct RAcc<true> {
  fvec4 re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
  __device__ __forceinline__ void mac(float2 a, float2 q) {
    re = mfma_f32(a.x, q.x, re);
    re = mfma_f32(a.y, q.y, re);
    im = mfma_f32(a.y, q.x, im);
    im = mfma_f32(-a.x, q.y, im);
  }
  __device__ __forceinline__ int row(int lane, int v) const { return f32_row(lane, v); }
  __device__ __forceinline__ void store(void* R, int64_t idx, int v, double sc = 1.0) const {
    float f = (float)sc;
    stg(reinterpret_cast<float2*>(R), idx, make_float2(re[v] * f, im[v] * f));
  }
};

// Column j of R^T: inherited columns in the level's arena, own-block
// columns (row basis) in the arena kept for the projection.  The item's
// fields are taken into registers once (the stores could alias the item
// array, so reading them at every store would reload them).
template <bool MX>
struct RDst {
  void* R;
  void* Rown;
  int64_t ninh;
  int k;
  __device__ __forceinline__ explicit RDst(const ItemDev& it)
      : R(it.R), Rown(it.Rown), ninh(it.ninh), k(it.k) {}
  __device__ __forceinline__ void* col(int64_t j) const {
    using E = typename std::conditional<MX, float2, double2>::type;
    return (Rown != nullptr && j >= ninh)
               ? static_cast<void*>(reinterpret_cast<E*>(Rown) + (j - ninh) * k)
               : static_cast<void*>(reinterpret_cast<E*>(R) + j * k);
  }
};

// Mixed form: largest |component| of the stored R values of tile t (rows
// kk = 16 t + lane % 16) into the workgroup's LDS maxima.
template <bool MX>
__device__ __forceinline__ void rmax_tile(const RAcc<MX>& acc, int64_t j0, int64_t ncols, int kk,
                                          int k, unsigned* s_rmax) {
  if constexpr (MX) {
    int lane = threadIdx.x & 63;
    float m = 0.0f;
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (j0 + acc.row(lane, v) < ncols) m = fmaxf(m, fmaxf(fabsf(acc.re[v]), fabsf(acc.im[v])));
    if (kk < k && m > 0.0f) atomicMax(s_rmax + kk, __float_as_uint(m));
  }
}

// Merge the workgroup's LDS maxima into it.rmax (after a barrier).
__device__ __forceinline__ void rmax_flush(const ItemDev& it, const unsigned* s_rmax) {
  for (int kk = threadIdx.x; kk < it.k; kk += blockDim.x)
    if (s_rmax[kk]) atomicMax(reinterpret_cast<unsigned*>(it.rmax) + kk, s_rmax[kk]);
}

// The rows of the product's operand: rows [0, k1) from P1 (column j at
// P1[j k1]) and rows [k1, r) from P2 (column j at P2[j k2]), both starting at
// column c0 (the sons' R of a non-leaf item).
struct RowsSrc {
  const void* P1;
  const void* P2;
  int k1, k2;
  int64_t c0;
};

// R^T of a block row read from memory, one workgroup per unit (column
// range): the four waves share Q_hat (in the compute precision, rows padded
// with zeros to r + 8) in LDS and take 16-column groups in turn.
// Non-leaf: R^T[j][kk] = zeta sum_rho [R_t1c'; R_t2c'][rho][j] conj(Q_hat[rho][kk]).
// Row rho of the operand is one load from the part that holds it.
// The operand values are loaded kRing - 1 k-steps ahead and Q_hat one step
// ahead, in rings of kRing register sets that are unrolled so that no loaded
// register is copied.
template <bool MX, int KT>
__device__ void rprod_rows_wg(const ItemDev& it, const RowsSrc& src, const UnitDev& u,
                              double zeta, const ROp<MX>* Qs, unsigned* s_rmax, int kc0 = 0) {
  using OT = ROp<MX>;
  using S = typename std::conditional<MX, float, double>::type;
  typedef S E2 __attribute__((ext_vector_type(2)));
  using GP = const __attribute__((address_space(1))) E2*;
  constexpr int kRing = 5;
  int w = wave_id(), lane = threadIdx.x & 63, row = lane & 15, kq = lane >> 4;
  const int r = it.r, k = it.k, k1 = src.k1, k2 = src.k2;
  const int nks = (r + 3) / 4;
  constexpr int ldq = 16 * KT;
  const int ncols = (int)u.ncols;
  const int64_t c0 = src.c0;
  const OT* R1 = reinterpret_cast<const OT*>(src.P1) + c0 * k1;  // column j at R1[j * k1]
  const OT* R2 = reinterpret_cast<const OT*>(src.P2) + c0 * k2;
  const RDst<MX> dst(it);
  for (int j0 = 16 * w; j0 < ncols; j0 += 64) {
    // one load per element: row rho of [R1; R2] in column j; columns past
    // the unit and rows past r read a valid element instead (their products
    // land in columns that are not stored, or meet zero rows of Q_hat)
    const int jc = min(j0 + row, ncols - 1);
    const OT* c1 = R1 + (int64_t)jc * k1;
    const OT* c2 = R2 + (int64_t)jc * k2 - k1;
    auto lda = [&](int rho, OT& a) {
      const int rc = min(rho, r - 1);
      E2 v = ((GP)(rc < k1 ? c1 + rc : c2 + rc))[0];
      a.x = v.x;
      a.y = v.y;
    };
    auto ldqs = [&](int rho, OT* q) {
#pragma unroll
      for (int t = 0; t < KT; ++t) q[t] = Qs[rho * ldq + 16 * t + row];
    };
    RAcc<MX> acc[KT];
    auto mac = [&](const OT& v, const OT* q) {
#pragma unroll
      for (int t = 0; t < KT; ++t) acc[t].mac(v, q[t]);
    };
    // ring of kRing register sets: son values kRing - 1 steps ahead, Q_hat
    // one step ahead
    OT a[kRing];
    OT q[kRing][KT];
    // drain the previous column group (stores, unused prefetches) so that the
    // wait counts inside the loop are exact
    __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
    for (int st = 0; st < kRing - 1; ++st) {
      lda(4 * st + kq, a[st]);
      __builtin_amdgcn_sched_barrier(0);
    }
    ldqs(kq, q[0]);
    int rho0 = 0;
    for (int n = nks / kRing; n > 0; --n, rho0 += 4 * kRing) {
#pragma unroll
      for (int st = 0; st < kRing; ++st) {
        lda(rho0 + 4 * (st + kRing - 1) + kq, a[(st + kRing - 1) % kRing]);
        ldqs(rho0 + 4 * (st + 1) + kq, q[(st + 1) % kRing]);
        __builtin_amdgcn_sched_barrier(0);
        mac(a[st], q[st]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int st = 0; st < kRing - 1; ++st) {
      if (st < nks % kRing) {
        ldqs(rho0 + 4 * (st + 1) + kq, q[(st + 1) % kRing]);
        mac(a[st], q[st]);
      }
    }
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      int kk = kc0 + 16 * t + row;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int64_t jv = j0 + acc[t].row(lane, v);
        if (jv < ncols && kk < k) acc[t].store(dst.col(u.col_begin + jv), kk, v, zeta);
      }
      if constexpr (MX) {
        // the stored values are the accumulators scaled by zeta in FP32
        RAcc<MX> sc = acc[t];
        float z = (float)zeta;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          sc.re[v] *= z;
          sc.im[v] *= z;
        }
        rmax_tile<MX>(sc, j0, ncols, kk, k, s_rmax);
      }
    }
  }
}

// every unit of one launch has ceil(k / 16) = KT
template <bool MX, int KT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MX && KT <= 3 ? 8 - 2 * KT + 2 : 1))) void k_rprod_inner_g(const ItemDev* items, const UnitDev* units,
                                                       double zeta) {
  extern __shared__ __align__(16) char rlds[];
  __shared__ unsigned s_rmax[kMaxR];
  using OT = ROp<MX>;
  OT* Qs = reinterpret_cast<OT*>(rlds);
  const UnitDev u = units[blockIdx.x];
  const ItemDev& it = items[u.item];
  const int r = it.r, k = it.k;
  if (k == 0 || (k + 15) / 16 != KT) return;
  constexpr int ldq = 16 * KT;
  for (int e = threadIdx.x; e < (r + 8) * ldq; e += 256) {
    int i = e / ldq, kk = e - i * ldq;
    Qs[e] = rop<MX>((i < r && kk < k) ? it.Q[(int64_t)i * k + kk] : make_double2(0.0, 0.0));
  }
  for (int kk = threadIdx.x; kk < kMaxR; kk += 256) s_rmax[kk] = 0u;
  __syncthreads();
  const ItemDev& s1 = items[it.son[0]];
  const ItemDev& s2 = items[it.son[1]];
  const RowsSrc src{s1.R, s2.R, s1.k, s2.k, it.col_off + u.col_begin};
  rprod_rows_wg<MX, KT>(it, src, u, zeta, Qs, s_rmax);
  if constexpr (MX) {
    __syncthreads();
    rmax_flush(it, s_rmax);
  }
}

// Large transfer factors (Q_hat beyond the LDS of one workgroup): Q_hat is
// packed into 64-column chunks in memory, (r + 8) x 64 each with zero rows
// and columns past r and k, and each unit forms the 64 columns of R^T of one
// chunk (unit field a0: the chunk index) for its column range.
template <bool MX>
__global__ __launch_bounds__(256) void k_rprod_inner_big(const ItemDev* items,
                                                         const UnitDev* units, double zeta,
                                                         const ROp<MX>* const* qchunk) {
  __shared__ unsigned s_rmax[kMaxRBig];
  const UnitDev u = units[blockIdx.x];
  const ItemDev& it = items[u.item];
  if (it.k == 0) return;
  for (int kk = threadIdx.x; kk < kMaxRBig; kk += 256) s_rmax[kk] = 0u;
  __syncthreads();
  const ItemDev& s1 = items[it.son[0]];
  const ItemDev& s2 = items[it.son[1]];
  const RowsSrc src{s1.R, s2.R, s1.k, s2.k, it.col_off + u.col_begin};
  rprod_rows_wg<MX, 4>(it, src, u, zeta, qchunk[blockIdx.x], s_rmax, 64 * u.a0);
  if constexpr (MX) {
    __syncthreads();
    rmax_flush(it, s_rmax);
  }
}

// Packs Q_hat of large transfer factors into the chunks read above: task q
// writes chunk c of item i (rows 0 .. r + 8, 64 columns) at dst.
__global__ __launch_bounds__(256) void k_pack_q(const ItemDev* items, const int32_t* item,
                                                const int32_t* chunk, void* const* dst,
                                                int mixed) {
  const ItemDev& it = items[item[blockIdx.x]];
  const int r = it.r, k = it.k, c0 = 64 * chunk[blockIdx.x];
  for (int e = threadIdx.x; e < (r + 8) * 64; e += 256) {
    int i = e >> 6, kk = c0 + (e & 63);
    double2 v = (i < r && kk < k) ? it.Q[(int64_t)i * k + kk] : make_double2(0.0, 0.0);
    if (mixed)
      reinterpret_cast<float2*>(dst[blockIdx.x])[e] = make_float2((float)v.x, (float)v.y);
    else
      reinterpret_cast<double2*>(dst[blockIdx.x])[e] = v;
  }
}

// R^T of a leaf block row: the workgroup's four waves share the item's factor
// Q (in LDS, compute precision) and take 16-column groups in turn.
template <int SRC, bool MX, int KT>
__device__ void rprod_leaf_wave(const GeomDev& g, const ItemDev& it, const EntDev* ents, int side,
                                const UnitDev& u, const ROp<MX>* Qs, const RowData* rows,
                                const double4* rown, unsigned* s_rmax) {
  // mixed form with generated entries: register-staged FP32 generators
  constexpr bool kGen = MX && (SRC == SRC_HELMHOLTZ || SRC == SRC_DLP);
  int w = wave_id(), lane = threadIdx.x & 63, row = lane & 15, kq = lane >> 4;
  int r = it.r, k = it.k;
  int nks = (r + 3) / 4;
  const RDst<MX> dst(it);
  const double4* const cols = it.cols;
  for (int64_t j0 = 16 * w; j0 < u.ncols; j0 += 64) {
    int64_t j = u.col_begin + j0 + row;
    double4 cc = kGen ? pad_col() : make_double4(0.0, 0.0, 0.0, 0.0);
    double4 cn = make_double4(0.0, 0.0, 0.0, 0.0);
    if (j0 + row < u.ncols) {
      cc = ldg(cols, j);
      if constexpr (kGen && SRC == SRC_DLP) cn = ldg(cols, it.N + j);
    }
    RAcc<MX> acc[KT];
    if constexpr (kGen) {
      // the lane's entries of all k-steps first (independent chains), then
      // the MFMAs (leaf block rows have at most 64 rows: 16 k-steps)
      float2 e[16];
#pragma unroll
      for (int ks = 0; ks < 16; ++ks)
        if (ks < nks) {
          if constexpr (SRC == SRC_HELMHOLTZ)
            e[ks] = gen_entry_mx(g, rows[4 * ks + kq], cc, side);
          else
            e[ks] = gen_entry_dlp_mx(g, rows[4 * ks + kq], rown[4 * ks + kq], cc, cn, side);
        }
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) {
        if (ks < nks) {
          int rho = 4 * ks + kq;
#pragma unroll
          for (int t = 0; t < KT; ++t) acc[t].mac(e[ks], Qs[rho * (16 * KT) + 16 * t + row]);
        }
      }
    } else {
      auto a = rop<MX>(gen_entry<SRC, MX>(g, rows[kq], cc, side));
      for (int ks = 0; ks < nks; ++ks) {
        int rho = 4 * ks + kq;
        // next k-step's entry (rows array is padded past r)
        auto an = rop<MX>(gen_entry<SRC, MX>(g, rows[rho + 4], cc, side));
#pragma unroll
        for (int t = 0; t < KT; ++t) acc[t].mac(a, Qs[rho * (16 * KT) + 16 * t + row]);
#pragma unroll
        for (int q = 0; q < 4 * KT; ++q) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);
        }
        a = an;
      }
    }
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      int kk = 16 * t + row;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int64_t jl = j0 + acc[t].row(lane, v);
        if (jl < u.ncols && kk < k) acc[t].store(dst.col(u.col_begin + jl), kk, v);
      }
      rmax_tile<MX>(acc[t], j0, u.ncols, kk, k, s_rmax);
    }
  }
}

template <int SRC, bool MX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MX ? 4 : 1))) void k_rprod_leaf_w(GeomDev g, const ItemDev* items,
                                                      const EntDev* ents, const UnitDev* units,
                                                      int side) {
  __shared__ ROp<MX> Qs[68 * 64];   // (r + 4) x (16 KT), zero padded rows past r
  __shared__ RowData rows[64 + 8];
  // mixed double layer: the rows' unit normals
  constexpr bool kDlpMx = MX && SRC == SRC_DLP;
  __shared__ double4 rown[kDlpMx ? 64 + 8 : 1];
  __shared__ unsigned s_rmax[64];
  const UnitDev u = units[blockIdx.x];
  const ItemDev& it = items[u.item];
  int r = it.r, k = it.k;
  if (k == 0) return;
  int kt = (k + 15) / 16;
  int ldq = 16 * kt;
  for (int e = threadIdx.x; e < (r + 4) * ldq; e += 256) {
    int i = e / ldq, kk = e - i * ldq;
    Qs[e] = rop<MX>((i < r && kk < k) ? it.Q[(int64_t)i * k + kk] : make_double2(0.0, 0.0));
  }
  for (int i = threadIdx.x; i < 72; i += 256) {
    // the mixed double layer stages positions like the single layer
    rows[i] = row_data<kDlpMx ? SRC_HELMHOLTZ : SRC>(g, it, i, side, MX);
    if constexpr (kDlpMx) rown[i] = row_normal(g, it, i);
  }
  for (int kk = threadIdx.x; kk < 64; kk += 256) s_rmax[kk] = 0u;
  __syncthreads();
  switch (kt) {
    case 1: rprod_leaf_wave<SRC, MX, 1>(g, it, ents, side, u, Qs, rows, rown, s_rmax); break;
    case 2: rprod_leaf_wave<SRC, MX, 2>(g, it, ents, side, u, Qs, rows, rown, s_rmax); break;
    case 3: rprod_leaf_wave<SRC, MX, 3>(g, it, ents, side, u, Qs, rows, rown, s_rmax); break;
    default: rprod_leaf_wave<SRC, MX, 4>(g, it, ents, side, u, Qs, rows, rown, s_rmax); break;
  }
  if constexpr (MX) {
    __syncthreads();
    rmax_flush(it, s_rmax);
  }
}

// ---------------------------------------------------------------------------
// Gram matrices of the mixed form on int8 MFMA (error-free slicing).
// Each real component x of row i of the block row is written as
//   x = 2^(E_i - 6) (d0 + d1 2^-8 + d2 2^-16 + d3 2^-24) + rest,
// with signed digits d in [-128, 127] of the truncated fixed-point value
// (balanced base 256) and E_i the exponent of a bound of the row's largest
// component over the unit, so |rest| < 2^(E_i - 30).  Products of digits
// accumulate exactly in int32 (16x16x64 MFMA); digit pairs with p + q <= 5
// (0-based) are kept (each dropped pair is below 2^-46 of the product of the
// row maxima per column), summed per p + q, and converted to FP64 once per
// unit.  The complex Gram A A^* = (Ar Ar^T + Ai Ai^T) + i (Ai Ar^T - Ar Ai^T)
// takes four real products per 16 x 16 tile pair.  One workgroup of 16 waves
// per unit: all threads generate (leaf) or load (non-leaf) and slice the
// next 64 columns into LDS while the waves run the MFMAs of the current 64
// columns.
// ---------------------------------------------------------------------------
typedef int ivec4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ ivec4 mfma_i8(ivec4 a, ivec4 b, ivec4 c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

constexpr int kI8Tiles = 6;                           // complex row tiles per unit
constexpr int kI8Threads = 1024;                      // 16 waves per unit
constexpr int kI8Waves = kI8Threads / 64;
constexpr int kI8ProdPerWave = 3;                     // 40 real tile products over 16 waves
constexpr int kI8Slab = 1024;                         // one slice of one tile: 16 rows x 64 B
constexpr int kI8Buf = kI8Tiles * 2 * 4 * kI8Slab;    // tiles x components x slices
constexpr size_t kI8Lds = 2 * (size_t)kI8Buf + 6 * 64 * sizeof(double4) +
                          kI8Tiles * 16 * (sizeof(RowData) + sizeof(double4) + 2 * sizeof(int));

__device__ __forceinline__ int i8_off(int T, int comp, int p, int g, int i) {
  return ((((T * 2 + comp) * 4 + p) * 4 + g) * 16 + i) * 16;
}

// Four int8 slices of 4 values, packed one dword each (out[p] holds slice p
// of value q in byte q; slice 0 is the most significant).  sc = 2^(30 - E)
// with |v| < 2^E, so Y = trunc(v sc) has |Y| < 2^30 and, in balanced base
// 256, Y = d0 2^24 + d1 2^16 + d2 2^8 + d3 exactly with digits in
// [-128, 127]: Z = Y + 0x808080 has the bytes z3 z2 z1 z0, the three low
// digits are z - 128 (the byte XOR 0x80) and the top digit is z3 read as a
// signed byte.  The bytes of the four Z are transposed with byte permutes.
__device__ __forceinline__ void i8_slice4(const float* v, float sc, unsigned* out) {
  unsigned z[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) z[q] = (unsigned)((int)(v[q] * sc) + 0x808080);
  // {z0.b0, z1.b0, z0.b1, z1.b1} and {z0.b2, z1.b2, z0.b3, z1.b3}, same for z2, z3
  const unsigned lo01 = __builtin_amdgcn_perm(z[1], z[0], 0x05010400u);
  const unsigned hi01 = __builtin_amdgcn_perm(z[1], z[0], 0x07030602u);
  const unsigned lo23 = __builtin_amdgcn_perm(z[3], z[2], 0x05010400u);
  const unsigned hi23 = __builtin_amdgcn_perm(z[3], z[2], 0x07030602u);
  // byte b of every value: {z0.bb, z1.bb, z2.bb, z3.bb}
  const unsigned b0 = __builtin_amdgcn_perm(lo23, lo01, 0x05040100u);
  const unsigned b1 = __builtin_amdgcn_perm(lo23, lo01, 0x07060302u);
  const unsigned b2 = __builtin_amdgcn_perm(hi23, hi01, 0x05040100u);
  const unsigned b3 = __builtin_amdgcn_perm(hi23, hi01, 0x07060302u);
  out[0] = b3;
  out[1] = b2 ^ 0x80808080u;
  out[2] = b1 ^ 0x80808080u;
  out[3] = b0 ^ 0x80808080u;
}

template <int KIND>  // 0: generated leaf block rows, 1: non-leaf block rows from the sons' R,
                     // 2: generated leaf block rows of the double layer
__global__ __launch_bounds__(kI8Threads) void k_gram_i8(GeomDev g, const ItemDev* items,
                                                 const EntDev* ents, const UnitDev* units,
                                                 int side, double zeta2, double2* partial) {
  extern __shared__ __align__(16) char lds[];
  char* slices = lds;
  double4* cold = reinterpret_cast<double4*>(lds + 2 * kI8Buf);  // 3 x 64 columns
  double4* coldn = cold + 3 * 64;  // double layer: their normals
  RowData* rowd = reinterpret_cast<RowData*>(coldn + 3 * 64);
  double4* rown = reinterpret_cast<double4*>(rowd + kI8Tiles * 16);  // double layer: row normals
  int* rexp = reinterpret_cast<int*>(rown + kI8Tiles * 16);
  unsigned* rmaxb = reinterpret_cast<unsigned*>(rexp + kI8Tiles * 16);

  const UnitDev u = units[blockIdx.x];
  const ItemDev& it = items[u.item];
  const int tid = threadIdx.x, w = wave_id(), lane = tid & 63;
  const bool diag = u.a0 == u.b0;
  const int na = u.na, nb = u.nb;
  const int ntile = diag ? na : na + nb;
  const int npair = diag ? na * (na + 1) / 2 : na * nb;
  const int nprod = 4 * npair;
  const int r = it.r;
  const int64_t ncols = u.ncols;
  const int nch = (int)((ncols + 63) >> 6);
  auto row0 = [&](int T) { return 16 * (T < na ? u.a0 + T : u.b0 + (T - na)); };

  // ---- row data and row bounds ----
  for (int e = tid; e < ntile * 16; e += kI8Threads) {
    rmaxb[e] = 0u;
    if constexpr (KIND != 1) {
      // positions and row factors (the double layer's too), padding far away
      rowd[e] = row_data<SRC_HELMHOLTZ>(g, it, row0(e >> 4) + (e & 15), side, true);
      if constexpr (KIND == 2) rown[e] = row_normal(g, it, row0(e >> 4) + (e & 15));
    }
  }
  auto stage_cols = [&](int c, int buf) {
    if constexpr (KIND != 1) {
      if (tid < 64) {
        int64_t j = (int64_t)c * 64 + tid;
        double4 v = pad_col(), vn = make_double4(0.0, 0.0, 0.0, 0.0);
        if (c < nch && j < ncols) {
          v = ldg(it.cols, u.col_begin + j);
          if constexpr (KIND == 2) vn = ldg(it.cols, it.N + u.col_begin + j);
        }
        cold[buf * 64 + tid] = v;
        if constexpr (KIND == 2) coldn[buf * 64 + tid] = vn;
      }
    }
  };
  __syncthreads();
  if constexpr (KIND == 2) {
    // double layer: the largest component of every row over the unit's
    // columns, from the entries themselves (a bound from the distances alone
    // overestimates these rows many times, since <x - y, n(y)> is much
    // smaller than |x - y| near the row point, and would waste slice bits)
    const int nrow = ntile * 16, stride = kI8Threads / nrow;
    if (tid < stride * nrow) {
      const int rl = tid % nrow;
      const RowData rw = rowd[rl];
      const double4 rn = rown[rl];
      float mx = 0.0f;
      if (rw.f != 0.0)
        for (int64_t j = tid / nrow; j < ncols; j += stride) {
          const float2 v = gen_entry_dlp_mx(g, rw, rn, ldg(it.cols, u.col_begin + j),
                                            ldg(it.cols, it.N + u.col_begin + j), side);
          mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
        }
      if (mx > 0.0f) atomicMax(&rmaxb[rl], __float_as_uint(mx));
    }
  } else if constexpr (KIND == 0) {
    // leaf rows: |entry| <= |f_i| scale_e wfac_e / (4 pi dist(x_i, box of s_e)) over
    // the column-set entries that meet the unit's column range
    __shared__ int64_t s_e0, s_e1;
    if (tid == 0) {
      int64_t lo = it.ent_begin, hi = it.ent_end - 1;
      while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (ents[mid].col_start <= u.col_begin) lo = mid;
        else hi = mid - 1;
      }
      s_e0 = lo;
      int64_t last = u.col_begin + ncols - 1;
      hi = it.ent_end - 1;
      while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (ents[mid].col_start <= last) lo = mid;
        else hi = mid - 1;
      }
      s_e1 = lo + 1;
    }
    __syncthreads();
    const int64_t e0 = s_e0, ne = s_e1 - s_e0;
    const int nrow = ntile * 16, stride = kI8Threads / nrow;
    if (tid < stride * nrow) {
      const int rl = tid % nrow;
      const RowData rw = rowd[rl];
      float mx = 0.0f;
      if (rw.f != 0.0) {
        for (int64_t q = tid / nrow; q < ne; q += stride) {
          const EntDev en = ents[e0 + q];
          const double* cb = g.cbox + 8 * en.s;
          double d2 = 0.0;
          double xs[3] = {rw.x, rw.y, rw.z};
#pragma unroll
          for (int a3 = 0; a3 < 3; ++a3) {
            double t = fmax(0.0, fmax(cb[a3] - xs[a3], xs[a3] - cb[3 + a3]));
            d2 += t * t;
          }
          // admissible blocks are separated from the row cluster, so d2 > 0
          double wf = side == 0 ? cb[6] : 1.0;
          mx = fmaxf(mx, (float)(fabs(rw.f) * en.scale * wf * kInv4Pi / sqrt(d2)));
        }
      }
      if (mx > 0.0f) atomicMax(&rmaxb[rl], __float_as_uint(mx));
    }
  } else {
    // non-leaf rows: the largest |component| of every row of the sons' R
    // (recorded by their R-products; a bound over any column range)
    for (int e = tid; e < ntile * 16; e += kI8Threads) {
      int rho = row0(e >> 4) + (e & 15);
      const ItemDev& s1 = items[it.son[0]];
      const ItemDev& s2 = items[it.son[1]];
      float m = 0.0f;
      if (rho < s1.k)
        m = s1.rmax[rho];
      else if (rho < r)
        m = s2.rmax[rho - s1.k];
      rmaxb[e] = __float_as_uint(m);
    }
  }
  __syncthreads();
  for (int e = tid; e < ntile * 16; e += kI8Threads) {
    float m = __uint_as_float(rmaxb[e]) * 1.01f;
    int E = m > 0.0f ? ilogbf(m) + 1 : -100000;
    rexp[e] = E > -100 ? E : -100000;   // rows below 2^-100 are taken as zero
  }
  __syncthreads();

  // ---- produce: entries of chunk c, sliced into buffer buf ----
  // non-leaf: the raw values of a chunk are loaded into registers one
  // iteration before they are sliced
  // combos of 4 columns: cb = ((T * 4 + gg) * 4 + pp) * 16 + i, columns
  // 16 gg + 4 pp .. + 3 of the chunk for row i of tile T
  // The loads of a combo are issued without branches: rows past r read row
  // r - 1 and columns past the unit its last column (all inside the sons'
  // R), and those values are then replaced by zeros.  Combos past the unit's
  // tiles (whole waves, since ntile * 256 is a multiple of 64) load nothing.
  float2 raw[2][4];
  auto load_raw = [&](int c) {
    if (c >= nch) return;
    const ItemDev& s1 = items[it.son[0]];
    const ItemDev& s2 = items[it.son[1]];
    const int k1 = s1.k;
    const int64_t c0 = it.col_off + u.col_begin;
#pragma unroll
    for (int h2 = 0; h2 < 2; ++h2) {
      const int cb = tid + kI8Threads * h2;
      if (cb >= ntile * 256) continue;
      const int i = cb & 15, pp = (cb >> 4) & 3, gg = (cb >> 6) & 3, T = cb >> 8;
      const int rho = row0(T) + i;
      const bool rowok = rho < r;
      const int rc = min(rho, r - 1);
      const bool first = rc < k1;
      const float2* src = first ? reinterpret_cast<const float2*>(s1.R) + rc
                                : reinterpret_cast<const float2*>(s2.R) + (rc - k1);
      const int64_t ld = first ? k1 : s2.k;
      const int64_t j0 = (int64_t)c * 64 + 16 * gg + 4 * pp;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t j = min(j0 + q, ncols - 1);
        const float2 v = ldg(src, (c0 + j) * ld);
        raw[h2][q] = rowok && j0 + q < ncols ? v : make_float2(0.0f, 0.0f);
      }
    }
  };
  auto produce = [&](int c, int buf) {
    char* S = slices + buf * kI8Buf;
#pragma unroll
    for (int h2 = 0; h2 < 2; ++h2) {
      int cb = tid + kI8Threads * h2;
      if (cb < ntile * 256) {
        int i = cb & 15, pp = (cb >> 4) & 3, gg = (cb >> 6) & 3, T = cb >> 8;
        int E = rexp[T * 16 + i];
        float sc = E > -100000 ? ldexpf(1.0f, 30 - E) : 0.0f;
        float vr[4], vi[4];
        if constexpr (KIND != 1) {
          const RowData rw = rowd[T * 16 + i];
          const double4* cc = cold + (c % 3) * 64 + 16 * gg + 4 * pp;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            float2 v;
            if constexpr (KIND == 0) {
              v = gen_entry_mx(g, rw, cc[q], side);
            } else {
              v = gen_entry_dlp_mx(g, rw, rown[T * 16 + i], cc[q],
                                   coldn[(c % 3) * 64 + 16 * gg + 4 * pp + q], side);
            }
            vr[q] = v.x;
            vi[q] = v.y;
          }
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            vr[q] = raw[h2][q].x;
            vi[q] = raw[h2][q].y;
          }
        }
        unsigned pr[4], pi[4];
        i8_slice4(vr, sc, pr);
        i8_slice4(vi, sc, pi);
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          *reinterpret_cast<unsigned*>(S + i8_off(T, 0, p, gg, i) + 4 * pp) = pr[p];
          *reinterpret_cast<unsigned*>(S + i8_off(T, 1, p, gg, i) + 4 * pp) = pi[p];
        }
      }
    }
  };

  ivec4 acc[kI8ProdPerWave][6];
#pragma unroll
  for (int s = 0; s < kI8ProdPerWave; ++s)
#pragma unroll
    for (int l = 0; l < 6; ++l) acc[s][l] = ivec4{0, 0, 0, 0};
  // product q = 4 pair + type; type 0: re re, 1: im im, 2: im re, 3: re im
  auto tiles_of = [&](int q, int& TA, int& TB, int& cA, int& cB) {
    int pair = q >> 2, type = q & 3;
    if (diag) {
      int I = 0;
      while ((I + 1) * (I + 2) / 2 <= pair) ++I;
      TA = I;
      TB = pair - I * (I + 1) / 2;
    } else {
      TA = pair / nb;
      TB = na + pair % nb;
    }
    cA = (type == 1 || type == 2) ? 1 : 0;
    cB = (type == 1 || type == 3) ? 1 : 0;
  };
  // LDS offsets of the wave's products, fixed over the chunks and the same
  // for all lanes of the wave: operand A of product s at offA[s] + 1024 p
  // (slice p) + 16 lane, operand B at offB[s] + 1024 q + 16 lane.  Taken
  // once for the non-leaf rows; the generated rows need those registers
  // for the entries and take them per chunk.
  int offA[kI8ProdPerWave], offB[kI8ProdPerWave];
  auto product_offsets = [&](int s) {
    offA[s] = offB[s] = 0;
    const int q = w + kI8Waves * s;
    if (q < nprod) {
      int TA, TB, cA, cB;
      tiles_of(q, TA, TB, cA, cB);
      offA[s] = __builtin_amdgcn_readfirstlane(i8_off(TA, cA, 0, 0, 0));
      offB[s] = __builtin_amdgcn_readfirstlane(i8_off(TB, cB, 0, 0, 0));
    }
  };
  if constexpr (KIND == 1) {
#pragma unroll
    for (int s = 0; s < kI8ProdPerWave; ++s) product_offsets(s);
  }
  auto consume = [&](int buf) {
    const char* S = slices + buf * kI8Buf + 16 * lane;
#pragma unroll
    for (int s = 0; s < kI8ProdPerWave; ++s) {
      int q = w + kI8Waves * s;
      if (q < nprod) {
        if constexpr (KIND != 1) product_offsets(s);
        // slice pairs (p, q) with p + q <= 5 (0-based) into level p + q
        ivec4 a[4];
#pragma unroll
        for (int p = 0; p < 4; ++p)
          a[p] = *reinterpret_cast<const ivec4*>(S + offA[s] + 1024 * p);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          ivec4 b = *reinterpret_cast<const ivec4*>(S + offB[s] + 1024 * q);
#pragma unroll
          for (int p = 0; p < 4; ++p)
            if (p + q <= 5) acc[s][p + q] = mfma_i8(a[p], b, acc[s][p + q]);
        }
      }
    }
  };

  // ---- pipeline over the chunks ----
  stage_cols(0, 0);
  stage_cols(1, 1);
  if constexpr (KIND == 1) load_raw(0);
  __syncthreads();
  produce(0, 0);
  if constexpr (KIND == 1) load_raw(1);
  __syncthreads();
  // waves w, w + 4, w + 8, w + 12 share a SIMD: half of them run the two
  // phases in the opposite order so that VALU work overlaps MFMAs
  const bool mfma_first = (w >> 2) & 1;
  for (int c = 0; c < nch; ++c) {
    stage_cols(c + 2, (c + 2) % 3);
    if (mfma_first) consume(c & 1);
    if (c + 1 < nch) produce(c + 1, (c + 1) & 1);
    if constexpr (KIND == 1) load_raw(c + 2);
    if (!mfma_first) consume(c & 1);
    __syncthreads();
  }

  // ---- FP64 conversion: real tile products to LDS, then complex pairs ----
  double* conv = reinterpret_cast<double*>(lds);  // nprod x 256, over the slice buffers
#pragma unroll
  for (int s = 0; s < kI8ProdPerWave; ++s) {
    int q = w + kI8Waves * s;
    if (q < nprod) {
      int TA, TB, cA, cB;
      tiles_of(q, TA, TB, cA, cB);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int row = 4 * (lane >> 4) + v, col = lane & 15;
        double x = 0.0;
#pragma unroll
        for (int l = 5; l >= 0; --l) x = x * 0.00390625 + (double)acc[s][l][v];
        int Ea = rexp[TA * 16 + row], Eb = rexp[TB * 16 + col];
        x = (Ea > -100000 && Eb > -100000) ? ldexp(x, Ea + Eb - 12) : 0.0;
        conv[q * 256 + row * 16 + col] = x;
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < npair * 256; e += kI8Threads) {
    int p = e >> 8, v = (e >> 6) & 3, l = e & 63;
    int row = (l >> 4) + 4 * v, col = l & 15, o = row * 16 + col;
    double re = conv[(4 * p) * 256 + o] + conv[(4 * p + 1) * 256 + o];
    double im = conv[(4 * p + 2) * 256 + o] - conv[(4 * p + 3) * 256 + o];
    partial[u.slot_off + e] = make_double2(re * zeta2, im * zeta2);
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_block_norm(int src, const GeomDev& g, const int64_t* t_off, const int64_t* t_len,
                       const int64_t* s_off, const int64_t* s_len, int64_t nblocks, double* omega,
                       hipStream_t st) {
  if (nblocks == 0) return;
  if (src == SRC_HELMHOLTZ)
    hipLaunchKernelGGL(k_block_norm<SRC_HELMHOLTZ>, dim3((unsigned)nblocks), dim3(256), 0, st, g,
                       t_off, t_len, s_off, s_len, nblocks, omega);
  else if (src == SRC_DLP)
    hipLaunchKernelGGL(k_block_norm<SRC_DLP>, dim3((unsigned)nblocks), dim3(256), 0, st, g,
                       t_off, t_len, s_off, s_len, nblocks, omega);
  else
    hipLaunchKernelGGL(k_block_norm<SRC_DENSE>, dim3((unsigned)nblocks), dim3(256), 0, st, g,
                       t_off, t_len, s_off, s_len, nblocks, omega);
}

void launch_block_norm2(int src, const GeomDev& g, const int64_t* t_off, const int64_t* t_len,
                        const int64_t* s_off, const int64_t* s_len, int64_t nblocks,
                        int max_iter, double tol, double* omega, hipStream_t st) {
  if (nblocks == 0) return;
  if (src == SRC_HELMHOLTZ)
    hipLaunchKernelGGL(k_block_norm2<SRC_HELMHOLTZ>, dim3((unsigned)nblocks), dim3(256), 0, st, g,
                       t_off, t_len, s_off, s_len, nblocks, max_iter, tol, omega);
  else if (src == SRC_DLP)
    hipLaunchKernelGGL(k_block_norm2<SRC_DLP>, dim3((unsigned)nblocks), dim3(256), 0, st, g,
                       t_off, t_len, s_off, s_len, nblocks, max_iter, tol, omega);
  else
    hipLaunchKernelGGL(k_block_norm2<SRC_DENSE>, dim3((unsigned)nblocks), dim3(256), 0, st, g,
                       t_off, t_len, s_off, s_len, nblocks, max_iter, tol, omega);
}

int block_norm2_max_size() { return kNorm2Max; }

void launch_entry_scale(EntDev* ent, int64_t nent, const double* omega, double zeta,
                        hipStream_t st) {
  if (nent == 0) return;
  hipLaunchKernelGGL(k_entry_scale, dim3(blocks_for(nent, 256)), dim3(256), 0, st, ent, nent,
                     omega, zeta);
}

void launch_gram(int src, bool inner, bool mixed, const GeomDev& g, const ItemDev* items,
                 const EntDev* ents, const UnitDev* units, int64_t nunits, double zeta, int side,
                 double2* partial, hipStream_t st) {
  if (nunits == 0) return;
  dim3 grid(blocks_for(nunits, 4)), blk(256);
  if (inner) {
    if (mixed)
      hipLaunchKernelGGL(k_gram_inner_w<true>, grid, blk, 0, st, items, units, nunits, zeta,
                         partial);
    else
      hipLaunchKernelGGL(k_gram_inner_w<false>, grid, blk, 0, st, items, units, nunits, zeta,
                         partial);
  } else if (src == SRC_HELMHOLTZ) {
    if (mixed)
      hipLaunchKernelGGL((k_gram_leaf_w<SRC_HELMHOLTZ, true>), grid, blk, 0, st, g, items, ents,
                         units, nunits, side, partial);
    else
      hipLaunchKernelGGL((k_gram_leaf_w<SRC_HELMHOLTZ, false>), grid, blk, 0, st, g, items, ents,
                         units, nunits, side, partial);
  } else if (src == SRC_DLP) {
    hipLaunchKernelGGL((k_gram_leaf_w<SRC_DLP, false>), grid, blk, 0, st, g, items, ents, units,
                       nunits, side, partial);
  } else {
    hipLaunchKernelGGL((k_gram_leaf_w<SRC_DENSE, false>), grid, blk, 0, st, g, items, ents, units,
                       nunits, side, partial);
  }
}

void launch_gram_reduce(const ItemDev* items, const int32_t* litems, int32_t nl,
                        const int32_t* ubegin, const UnitDev* units, const double2* partial,
                        hipStream_t st) {
  if (nl == 0) return;
  hipLaunchKernelGGL(k_gram_reduce, dim3(nl), dim3(256), 0, st, items, litems, ubegin, units,
                     partial);
}

void launch_ranks(const ItemDev* items, int32_t n, int32_t* out, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_ranks, dim3(blocks_for(n, 256)), dim3(256), 0, st, items, n, out);
}

void launch_factor(ItemDev* items, const int32_t* litems, int32_t nl, int32_t rmax, double eps,
                   int max_sweeps, int32_t* status, hipStream_t st, bool wide) {
  if (nl == 0) return;
  static std::once_flag attr;
  std::call_once(attr, [] {
    (void)hipFuncSetAttribute((const void*)k_factor<kMaxR, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(kEigLds * sizeof(double2)));
  });
  // X needs p columns (the numerical rank of the Gram matrix above the cut),
  // plus one for the even pairing.  First pass: X within kFacLdsX elements
  // (two workgroups per CU) even where that holds fewer than r + 1 columns;
  // a factor that needs more is marked and factored again with room for all
  // columns (wide: up to kEigLds, one workgroup per CU)
  const int full = std::max(2, rmax * (rmax + 1));
  int cap = wide ? std::min(kEigLds, full) : std::min(kFacLdsX, full);
  hipLaunchKernelGGL((k_factor<kMaxR, false>), dim3(nl), dim3(kFacThreads),
                     (size_t)cap * sizeof(double2), st, items, litems, eps, max_sweeps, cap,
                     status, nullptr);
}

void launch_factor_big(ItemDev* items, const int32_t* litems, int32_t nl, double eps,
                       int max_sweeps, int32_t* status, double2* const* xptr, hipStream_t st) {
  if (nl == 0) return;
  // X of item q at xptr[q] with room for r (r + 1) elements: all r columns
  hipLaunchKernelGGL((k_factor<kMaxRBig, true>), dim3(nl), dim3(kFacThreads), 0, st, items,
                     litems, eps, max_sweeps, kMaxRBig * (kMaxRBig + 1), status, xptr);
}

void launch_leaf_cols(int src, const GeomDev& g, const ItemDev* items, const int32_t* litems,
                      int32_t nl, const EntDev* ents, int side, bool mixed, hipStream_t st) {
  if (nl == 0) return;
  if (src == SRC_HELMHOLTZ)
    hipLaunchKernelGGL(k_leaf_cols<SRC_HELMHOLTZ>, dim3(nl), dim3(256), 0, st, g, items, litems,
                       ents, side, 0);
  else if (src == SRC_DLP)
    hipLaunchKernelGGL(k_leaf_cols<SRC_DLP>, dim3(nl), dim3(256), 0, st, g, items, litems, ents,
                       side, mixed ? 1 : 0);
  else
    hipLaunchKernelGGL(k_leaf_cols<SRC_DENSE>, dim3(nl), dim3(256), 0, st, g, items, litems, ents,
                       side, 0);
}

void launch_gram_i8(bool inner, const GeomDev& g, const ItemDev* items, const EntDev* ents,
                    const UnitDev* units, int64_t nunits, double zeta, int side, double2* partial,
                    hipStream_t st, bool dlp) {
  if (nunits == 0) return;
  static std::once_flag attr;
  std::call_once(attr, [] {
    (void)hipFuncSetAttribute((const void*)k_gram_i8<0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)kI8Lds);
    (void)hipFuncSetAttribute((const void*)k_gram_i8<1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)kI8Lds);
    (void)hipFuncSetAttribute((const void*)k_gram_i8<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)kI8Lds);
  });
  if (inner)
    hipLaunchKernelGGL(k_gram_i8<1>, dim3((unsigned)nunits), dim3(kI8Threads), kI8Lds, st, g, items,
                       ents, units, side, zeta * zeta, partial);
  else if (dlp)
    hipLaunchKernelGGL(k_gram_i8<2>, dim3((unsigned)nunits), dim3(kI8Threads), kI8Lds, st, g, items,
                       ents, units, side, 1.0, partial);
  else
    hipLaunchKernelGGL(k_gram_i8<0>, dim3((unsigned)nunits), dim3(kI8Threads), kI8Lds, st, g, items,
                       ents, units, side, 1.0, partial);
}

size_t rprod_inner_lds_max() { return kRprodLdsMax; }

size_t rprod_inner_lds(bool mixed, int r, int k) {
  int kt = (k + 15) / 16;
  return (size_t)(r + 8) * 16 * kt * (mixed ? sizeof(float2) : sizeof(double2));
}

template <bool MX, int KT>
static void launch_rpi(const ItemDev* items, const UnitDev* units, int64_t nunits, double zeta,
                       size_t lds, hipStream_t st) {
  static std::once_flag attr;
  std::call_once(attr, [] {
    (void)hipFuncSetAttribute((const void*)k_rprod_inner_g<MX, KT>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRprodLdsMax);
  });
  hipLaunchKernelGGL((k_rprod_inner_g<MX, KT>), dim3((unsigned)nunits), dim3(256), lds, st, items,
                     units, zeta);
}

template <bool MX>
static void launch_rpi_kt(int kt, const ItemDev* items, const UnitDev* units, int64_t nunits,
                          double zeta, size_t lds, hipStream_t st) {
  switch (kt) {
    case 1: launch_rpi<MX, 1>(items, units, nunits, zeta, lds, st); break;
    case 2: launch_rpi<MX, 2>(items, units, nunits, zeta, lds, st); break;
    case 3: launch_rpi<MX, 3>(items, units, nunits, zeta, lds, st); break;
    case 4: launch_rpi<MX, 4>(items, units, nunits, zeta, lds, st); break;
    case 5: launch_rpi<MX, 5>(items, units, nunits, zeta, lds, st); break;
    case 6: launch_rpi<MX, 6>(items, units, nunits, zeta, lds, st); break;
    case 7: launch_rpi<MX, 7>(items, units, nunits, zeta, lds, st); break;
    default: launch_rpi<MX, 8>(items, units, nunits, zeta, lds, st); break;
  }
}

void launch_rprod_leaf(int src, bool mixed, const GeomDev& g, const ItemDev* items,
                       const EntDev* ents, const UnitDev* units, int64_t nunits, int side,
                       hipStream_t st) {
  if (nunits == 0) return;
  dim3 blk(256), grid((unsigned)nunits);
  if (src == SRC_HELMHOLTZ) {
    if (mixed)
      hipLaunchKernelGGL((k_rprod_leaf_w<SRC_HELMHOLTZ, true>), grid, blk, 0, st, g, items, ents,
                         units, side);
    else
      hipLaunchKernelGGL((k_rprod_leaf_w<SRC_HELMHOLTZ, false>), grid, blk, 0, st, g, items, ents,
                         units, side);
  } else if (src == SRC_DLP) {
    if (mixed)
      hipLaunchKernelGGL((k_rprod_leaf_w<SRC_DLP, true>), grid, blk, 0, st, g, items, ents,
                         units, side);
    else
      hipLaunchKernelGGL((k_rprod_leaf_w<SRC_DLP, false>), grid, blk, 0, st, g, items, ents,
                         units, side);
  } else {
    hipLaunchKernelGGL((k_rprod_leaf_w<SRC_DENSE, false>), grid, blk, 0, st, g, items, ents,
                       units, side);
  }
}

void launch_rprod_inner(bool mixed, int kt, const ItemDev* items, const UnitDev* units,
                        int64_t nunits, double zeta, size_t lds, hipStream_t st) {
  if (nunits == 0) return;
  if (mixed)
    launch_rpi_kt<true>(kt, items, units, nunits, zeta, lds, st);
  else
    launch_rpi_kt<false>(kt, items, units, nunits, zeta, lds, st);
}

void launch_pack_q(const ItemDev* items, const int32_t* item, const int32_t* chunk,
                   void* const* dst, int64_t ntasks, bool mixed, hipStream_t st) {
  if (ntasks == 0) return;
  hipLaunchKernelGGL(k_pack_q, dim3((unsigned)ntasks), dim3(256), 0, st, items, item, chunk, dst,
                     mixed ? 1 : 0);
}

void launch_rprod_inner_big(bool mixed, const ItemDev* items, const UnitDev* units,
                            int64_t nunits, double zeta, const void* const* qchunk,
                            hipStream_t st) {
  if (nunits == 0) return;
  if (mixed)
    hipLaunchKernelGGL(k_rprod_inner_big<true>, dim3((unsigned)nunits), dim3(256), 0, st, items,
                       units, zeta, (const float2* const*)qchunk);
  else
    hipLaunchKernelGGL(k_rprod_inner_big<false>, dim3((unsigned)nunits), dim3(256), 0, st, items,
                       units, zeta, (const double2* const*)qchunk);
}

void launch_expand(const ExpandDev* tasks, int64_t ntasks, hipStream_t st) {
  if (ntasks == 0) return;
  hipLaunchKernelGGL(k_expand, dim3((unsigned)ntasks), dim3(256), 0, st, tasks);
}

void launch_cvt(const CvtDev* tasks, int64_t ntasks, hipStream_t st) {
  if (ntasks == 0) return;
  hipLaunchKernelGGL(k_cvt, dim3((unsigned)ntasks), dim3(256), 0, st, tasks);
}

void launch_copy_c(const double2* src, int64_t src_off, double2* dst, int64_t dst_off,
                   int64_t count, hipStream_t st) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_copy_c, dim3(blocks_for(count, 256)), dim3(256), 0, st, src, src_off, dst,
                     dst_off, count);
}

void launch_project_stacked(int nc, const PTileDev* tiles, int64_t ntiles, const PBlkDev* blks,
                            const double* omega, hipStream_t st) {
  if (ntiles == 0) return;
  dim3 grid((unsigned)((ntiles + 3) / 4));
#define DH2_PST_NC(C)                                                                      \
  case C:                                                                                  \
    hipLaunchKernelGGL((k_project_stacked<C, (C <= 6 ? 4 : C <= 9 ? 3 : 2)>), grid,       \
                       dim3(256), 0, st, tiles, ntiles, blks, omega);                      \
    break;
  switch (nc) {
    DH2_PST_NC(1) DH2_PST_NC(2) DH2_PST_NC(3) DH2_PST_NC(4)
    DH2_PST_NC(5) DH2_PST_NC(6) DH2_PST_NC(7) DH2_PST_NC(8)
    DH2_PST_NC(9) DH2_PST_NC(10) DH2_PST_NC(11) DH2_PST_NC(12)
    DH2_PST_NC(13) DH2_PST_NC(14) DH2_PST_NC(15) DH2_PST_NC(16)
    default: break;
  }
#undef DH2_PST_NC
}

void launch_project(bool mixed, const ProjDev* tasks, int64_t ntasks, const double* omega,
                    hipStream_t st) {
  if (ntasks == 0) return;
  if (mixed)
    hipLaunchKernelGGL(k_project<true>, dim3(blocks_for(ntasks, 4)), dim3(256), 0, st, tasks,
                       ntasks, omega);
  else
    hipLaunchKernelGGL(k_project<false>, dim3(blocks_for(ntasks, 4)), dim3(256), 0, st, tasks,
                       ntasks, omega);
}

int project_rows_per_pass(bool mixed, int ntj) { return (mixed || ntj <= 2) ? 4 : 2; }

template <bool MX, int NJ, int SPLIT>
static void launch_pt(int ni, const ProjDev* tasks, int64_t ntasks, const double* omega,
                      hipStream_t st) {
  // row tiles per pass allowed by the register budget (project_rows_per_pass)
  constexpr int MAXI = (MX || NJ <= 2) ? 4 : 2;
  dim3 grid(SPLIT > 1 ? (unsigned)ntasks : blocks_for(ntasks, 4)), blk(256);
  switch (ni) {
    case 1: hipLaunchKernelGGL((k_project_tiled<MX, 1, NJ, SPLIT>), grid, blk, 0, st, tasks, ntasks, omega); break;
    case 2: hipLaunchKernelGGL((k_project_tiled<MX, 2, NJ, SPLIT>), grid, blk, 0, st, tasks, ntasks, omega); break;
    case 3:
      if constexpr (MAXI >= 3)
        hipLaunchKernelGGL((k_project_tiled<MX, 3, NJ, SPLIT>), grid, blk, 0, st, tasks, ntasks, omega);
      break;
    default:
      if constexpr (MAXI >= 4)
        hipLaunchKernelGGL((k_project_tiled<MX, 4, NJ, SPLIT>), grid, blk, 0, st, tasks, ntasks, omega);
      break;
  }
}

template <bool MX, int SPLIT>
static void launch_pt_nj(int ni, int nj, const ProjDev* tasks, int64_t ntasks,
                         const double* omega, hipStream_t st) {
  switch (nj) {
    case 1: launch_pt<MX, 1, SPLIT>(ni, tasks, ntasks, omega, st); break;
    case 2: launch_pt<MX, 2, SPLIT>(ni, tasks, ntasks, omega, st); break;
    case 3: launch_pt<MX, 3, SPLIT>(ni, tasks, ntasks, omega, st); break;
    default: launch_pt<MX, 4, SPLIT>(ni, tasks, ntasks, omega, st); break;
  }
}

void launch_project_tiled(bool mixed, int ni, int nj, bool split, const ProjDev* tasks,
                          int64_t ntasks, const double* omega, hipStream_t st) {
  if (ntasks == 0) return;
  if (mixed) {
    if (split) launch_pt_nj<true, 4>(ni, nj, tasks, ntasks, omega, st);
    else launch_pt_nj<true, 1>(ni, nj, tasks, ntasks, omega, st);
  } else {
    if (split) launch_pt_nj<false, 4>(ni, nj, tasks, ntasks, omega, st);
    else launch_pt_nj<false, 1>(ni, nj, tasks, ntasks, omega, st);
  }
}

void launch_near(int src, const GeomDev& g, const int64_t* t_off, const int64_t* t_len,
                 const int64_t* s_off, const int64_t* s_len, const int64_t* out_off,
                 int64_t nblocks, void* out, int f32, hipStream_t st) {
  if (nblocks == 0) return;
  auto go = [&](auto tag) {
    using SE = decltype(tag);
    SE* o = static_cast<SE*>(out);
    if (src == SRC_HELMHOLTZ)
      hipLaunchKernelGGL((k_near<SRC_HELMHOLTZ, SE>), dim3((unsigned)nblocks), dim3(256), 0, st, g,
                         t_off, t_len, s_off, s_len, out_off, o);
    else if (src == SRC_DLP)
      hipLaunchKernelGGL((k_near<SRC_DLP, SE>), dim3((unsigned)nblocks), dim3(256), 0, st, g, t_off,
                         t_len, s_off, s_len, out_off, o);
    else
      hipLaunchKernelGGL((k_near<SRC_DENSE, SE>), dim3((unsigned)nblocks), dim3(256), 0, st, g,
                         t_off, t_len, s_off, s_len, out_off, o);
  };
  if (f32)
    go(float2{});
  else
    go(double2{});
}

// Scratch memory of the allocation-free matrix-vector product: one array per
// device (its own copy on every GPU the library runs on), held until the
// process ends.  Host code uses the device address returned by
// noalloc_scratch(), never the array's name.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

size_t noalloc_scratch_bytes() { return kScratchBytes; }

hipError_t noalloc_scratch(void** out) {
  constexpr int kMaxDev = 64;
  static std::mutex mu;
  static void* addr[kMaxDev] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *out = addr[dev];
  return hipSuccess;
}

void launch_gather_perm(const double2* x, const int64_t* perm, int64_t n, double2* xp,
                        hipStream_t st, int nr) {
  hipLaunchKernelGGL(k_gather_perm, dim3(blocks_for(n, 256)), dim3(256), 0, st, x, perm, n, nr,
                     xp);
}
void launch_scatter_perm(const double2* yp, const int64_t* perm, int64_t n, double2* y,
                         hipStream_t st, int nr) {
  hipLaunchKernelGGL(k_scatter_perm, dim3(blocks_for(n, 256)), dim3(256), 0, st, yp, perm, n, nr,
                     y);
}

// the right-hand-side bound of the kernel instance: 1, 2, 4 or 8
#define DH2_NR_DISPATCH(nr, ...)                        \
  do {                                                  \
    if ((nr) <= 1) {                                    \
      constexpr int NR = 1;                             \
      __VA_ARGS__;                                      \
    } else if ((nr) <= 2) {                             \
      constexpr int NR = 2;                             \
      __VA_ARGS__;                                      \
    } else if ((nr) <= 4) {                             \
      constexpr int NR = 4;                             \
      __VA_ARGS__;                                      \
    } else {                                            \
      constexpr int NR = 8;                             \
      __VA_ARGS__;                                      \
    }                                                   \
  } while (0)

void launch_fwd_leaf(const ItemDev* items, const int32_t* litems, int32_t nl,
                     const int64_t* xh_off, const double2* xp, double2* xh, int nr,
                     hipStream_t st) {
  if (nl == 0) return;
  DH2_NR_DISPATCH(nr, hipLaunchKernelGGL(k_fwd_leaf<NR>, dim3(nl), dim3(128), 0, st, items, litems,
                                         xh_off, xp, xh, nr));
}
void launch_fwd_inner(const ItemDev* items, const int32_t* litems, int32_t nl,
                      const int64_t* xh_off, double2* xh, int nr, hipStream_t st) {
  if (nl == 0) return;
  DH2_NR_DISPATCH(nr, hipLaunchKernelGGL(k_fwd_inner<NR>, dim3(nl), dim3(128), 0, st, items,
                                         litems, xh_off, xh, nr));
}
// S_b^T of every admissible block (one workgroup per block)
template <typename SE>
__global__ __launch_bounds__(256) void k_coupling_transpose(const void* const* S,
                                                            void* const* ST,
                                                            const int32_t* rows,
                                                            const int32_t* cols) {
  const int b = blockIdx.x;
  const SE* A = static_cast<const SE*>(S[b]);
  SE* T = static_cast<SE*>(ST[b]);
  const int kr = rows[b], kc = cols[b];
  for (int e = threadIdx.x; e < kr * kc; e += 256) {
    const int i = e % kr, j = e / kr;
    T[j + (int64_t)i * kc] = A[e];
  }
}

void launch_coupling_transpose(const void* const* S, void* const* ST, const int32_t* rows,
                               const int32_t* cols, int64_t nblocks, int f32, hipStream_t st) {
  if (nblocks == 0) return;
  if (f32)
    hipLaunchKernelGGL(k_coupling_transpose<float2>, dim3((unsigned)nblocks), dim3(256), 0, st, S,
                       ST, rows, cols);
  else
    hipLaunchKernelGGL(k_coupling_transpose<double2>, dim3((unsigned)nblocks), dim3(256), 0, st, S,
                       ST, rows, cols);
}

void launch_coupling(const ItemDev* items, int32_t nitems, int32_t nheavy,
                     const int32_t* order, const int64_t* cbegin, const int32_t* cblock,
                     const int32_t* cpartner, const void* const* S_ptr,
                     const int32_t* S_rows, const int32_t* S_cols, const int64_t* xh_off,
                     const double2* xh, const int64_t* yh_off, double2* yh, int adjoint, int nr,
                     int f32, hipStream_t st) {
  if (nitems == 0) return;
  // one launch: workgroups [0, nheavy) one item each, then four items each
  const int32_t nwg = nheavy + (nitems - nheavy + 3) / 4;
  if (f32)
    DH2_NR_DISPATCH(nr, hipLaunchKernelGGL((k_coupling<NR, float2>), dim3(nwg), dim3(256), 0, st,
                                           items, nitems, nheavy, order, cbegin, cblock, cpartner,
                                           S_ptr, S_rows, S_cols, xh_off, xh, yh_off, yh, adjoint,
                                           nr));
  else
    DH2_NR_DISPATCH(nr, hipLaunchKernelGGL((k_coupling<NR, double2>), dim3(nwg), dim3(256), 0, st,
                                           items, nitems, nheavy, order, cbegin, cblock, cpartner,
                                           S_ptr, S_rows, S_cols, xh_off, xh, yh_off, yh, adjoint,
                                           nr));
}
void launch_bwd_inner(const ItemDev* items, const int32_t* litems, int32_t nl,
                      const int64_t* fbegin, const int32_t* fitem, const int32_t* fsonidx,
                      const int64_t* yh_off, double2* yh, int nr, hipStream_t st) {
  if (nl == 0) return;
  DH2_NR_DISPATCH(nr, hipLaunchKernelGGL(k_bwd_inner<NR>, dim3(nl), dim3(128), 0, st, items,
                                         litems, fbegin, fitem, fsonidx, yh_off, yh, nr));
}
void launch_bwd_leaf(const ItemDev* items, const LeafDev* leaves, int32_t nleaves,
                     const NearRefDev* nref, const NearDev* nears, const void* nearv,
                     const void* nearT, const int64_t* yh_off, const double2* yh,
                     const double2* xp, double2* yp, double2* partial, int adjoint, int nr,
                     int near, int accumulate, int f32, hipStream_t st) {
  if (nleaves == 0) return;
  if (near && f32)
    DH2_NR_DISPATCH(nr, hipLaunchKernelGGL((k_bwd_leaf<NR, true, float2>), dim3(nleaves),
                                           dim3(256), 0, st, items, leaves, nref, nears, nearv,
                                           nearT, yh_off, yh, xp, yp, partial, adjoint, nr,
                                           accumulate));
  else if (near)
    DH2_NR_DISPATCH(nr, hipLaunchKernelGGL((k_bwd_leaf<NR, true, double2>), dim3(nleaves),
                                           dim3(256), 0, st, items, leaves, nref, nears, nearv,
                                           nearT, yh_off, yh, xp, yp, partial, adjoint, nr,
                                           accumulate));
  else
    DH2_NR_DISPATCH(nr, hipLaunchKernelGGL((k_bwd_leaf<NR, false, double2>), dim3(nleaves),
                                           dim3(256), 0, st, items, leaves, nref, nears, nearv,
                                           nearT, yh_off, yh, xp, yp, partial, adjoint, nr,
                                           accumulate));
}

void launch_leaf_sum(const LeafDev* leaves, int32_t nleaves, const double2* partial, double2* yp,
                     int nr, hipStream_t st) {
  if (nleaves == 0) return;
  DH2_NR_DISPATCH(nr, hipLaunchKernelGGL(k_leaf_sum<NR>, dim3(nleaves), dim3(64), 0, st, leaves,
                                         partial, yp, nr));
}

void launch_near_transpose(const NearDev* nears, int64_t nblocks, const void* B, void* BT,
                           int f32, hipStream_t st) {
  if (nblocks == 0) return;
  if (f32)
    hipLaunchKernelGGL(k_near_transpose<float2>, dim3((unsigned)nblocks), dim3(256), 0, st, nears,
                       static_cast<const float2*>(B), static_cast<float2*>(BT));
  else
    hipLaunchKernelGGL(k_near_transpose<double2>, dim3((unsigned)nblocks), dim3(256), 0, st, nears,
                       static_cast<const double2*>(B), static_cast<double2*>(BT));
}
void launch_direct(int src, const GeomDev& g, const int64_t* rows, int64_t nrows,
                   const double2* xp, int adjoint, double2* out, hipStream_t st) {
  if (nrows == 0) return;
  if (src == SRC_HELMHOLTZ)
    hipLaunchKernelGGL(k_direct<SRC_HELMHOLTZ>, dim3((unsigned)nrows), dim3(256), 0, st, g, rows,
                       nrows, xp, adjoint, out);
  else if (src == SRC_DLP)
    hipLaunchKernelGGL(k_direct<SRC_DLP>, dim3((unsigned)nrows), dim3(256), 0, st, g, rows,
                       nrows, xp, adjoint, out);
  else
    hipLaunchKernelGGL(k_direct<SRC_DENSE>, dim3((unsigned)nrows), dim3(256), 0, st, g, rows,
                       nrows, xp, adjoint, out);
}

}  // namespace dh2
