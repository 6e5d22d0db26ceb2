// Device-side building blocks shared by the DPDE kernels: system descriptors,
// the counter-based pair noise, box geometry and deterministic reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace dpde {

constexpr int kWave = 64;

// Device status word bits (sticky for the rest of a dpde_step call).
enum : uint32_t {
  ST_NEG_EINT = 1u,   // eps_i <= 0 or T_i <= 0
  ST_OVERFLOW = 2u,   // neighbour list capacity exceeded
  ST_NONFINITE = 4u,  // NaN/Inf in positions or momenta
  ST_EOS = 8u,        // temperature inversion failed
  ST_RANGE = 16u,     // a pair term outside the range of the fixed-point pair sums
};

// Geometry and noise key of one system (replica).
struct Geo {
  double box[3];
  double half_box[3];
  double scale[3];     // cells per unit length: nc / box
  int32_t nc[3];
  int32_t periodic[3];
  int64_t cell_base;   // global index of the replica's cell 0
  int64_t first;       // first row (identifier space) of the replica
  int64_t n;           // particles in the replica
  uint32_t key0, key1; // Philox key: seed low word, seed high word ^ replica
  double dscale[3];    // Hybrid domains per unit length: ndom / box
  int32_t ndom[3];     // Hybrid domains per dimension
  int32_t oblk;        // edge (in cells) of the cell blocks of the memory order
  float oblk_inv;      // 1 / oblk (FP32)
  int64_t dom_base;    // global index of the replica's domain 0
};

// A kernel's view of its replica's geometry: batched kernels (one replica
// per particle, so the fields differ across a wave) hold a copy in registers,
// because through a reference the compiler reloads the fields after every
// global store in their pair loops; single-system kernels keep a reference,
// whose uniform fields load into scalar registers.
template <bool BATCH>
using GeoRef = std::conditional_t<BATCH, Geo, const Geo&>;

// Physical parameters shared by all replicas of a handle.
struct Phys {
  double mass, inv_mass, inv_2m;
  double rc, inv_rc, rc2;
  double a, half_a_rc;      // force amplitude, potential prefactor a rc / 2
  double gkT_half;          // gamma kT_ref / 2: gamma_ij = gkT_half (1/T_i + 1/T_j)
  double sigma, dt, half_dt, sqrt_dt;
  double dsigma2_m;         // k sigma^2 / m with k noise dimensions (SEM drift)
  double cv, eos_n, eos_omega, eos_c0;
  double mlp_in_c, mlp_in_s, mlp_out_c, mlp_out_s, mlp_eps_lo, mlp_eps_hi;
  // splined LJ: v = c12/r^12 - c6/r^6 - v_c - dv_c (r - rc), r_lj2 = r_lj^2
  double lj4e, r_lj2, lj_vc, lj_dvc;
  // farthest a listed neighbour can be: rc + 2 skin (built within rc + skin,
  // each particle moves at most skin/2 before the next build)
  double reach;
  int32_t eos, theta_mode, precision, scheme;
  int32_t cap;              // neighbour list capacity per particle
  int32_t model;            // 0: along v_ij (3-d G), 1: along e_ij (scalar xi)
  int32_t potential;        // 0: soft, 1: splined LJ
  int32_t project;          // eps projection after every step
  // tile form, pass A: grid 2^-g of the force and potential sums, chosen so
  // that every soft-potential term (|f d| <= a, v/2 <= a rc/4) stays below
  // 2^(51-g) / 2; fix_ok = 0 when no grid down to 2^-30 does (the tile form
  // is then not used)
  double fix_scale_f, fix_inv_f;
  int32_t fix_ok;
  int32_t pad_fix;
};

// -------------------------------------------------------------------------
// Pair noise G_ij^n: Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// with counter (lo id, hi id, n_lo, n_hi) and the replica key, then
// Box-Muller.  The noise is a pure function of (key, lo, hi, n), which is
// what lets the second SER sweep regenerate the first sweep's increments
// (Sec. 3.2.1).
// -------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t& x0, uint32_t& x1, uint32_t& x2,
                                              uint32_t& x3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t m0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    const uint64_t m1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    const uint32_t y0 = (uint32_t)(m1 >> 32) ^ x1 ^ k0;
    const uint32_t y2 = (uint32_t)(m0 >> 32) ^ x3 ^ k1;
    x1 = (uint32_t)m1;
    x3 = (uint32_t)m0;
    x0 = y0;
    x2 = y2;
  }
}

__device__ __forceinline__ void pair_words(const Geo& g, uint32_t lo, uint32_t hi, uint64_t step,
                                           uint32_t w[4]) {
  w[0] = lo;
  w[1] = hi;
  w[2] = (uint32_t)step;
  w[3] = (uint32_t)(step >> 32);
  philox4x32_10(w[0], w[1], w[2], w[3], g.key0, g.key1);
}

// ---------------------------------------------------------------------------
// FP64 elementary functions for the Box-Muller transform, specialised to its
// arguments and written from their series (relative error a few units in the
// last place, against ~100 instructions for the general library logarithm).
// ---------------------------------------------------------------------------

// ln u for u = (x + 1/2) 2^-32 = (2x + 1) 2^-33.  With 2x + 1 = m 2^e and
// m in [1/sqrt 2, sqrt 2): ln u = (e - 33) ln 2 + ln m, and
// ln m = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...), s = (m - 1)/(m + 1),
// |s| <= 0.172 (eleven terms leave a relative remainder below 1e-18).
__device__ __forceinline__ double ln_uniform_f64(uint32_t x) {
  const double y = 2.0 * (double)x + 1.0;  // exact
  double m = __builtin_amdgcn_frexp_mant(y);  // [1/2, 1)
  int e = __builtin_amdgcn_frexp_exp(y);
  if (m < 0.70710678118654752) {
    m *= 2.0;
    e -= 1;
  }
  const double f = m - 1.0;  // exact
  const double d = m + 1.0;
  // s = f / d: reciprocal seed, one Newton step, one residual correction
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  double s = f * r;
  s = fma(r, fma(-s, d, f), s);
  const double z = s * s;
  double p = 0.09523809523809523;  // 2/21
  p = fma(p, z, 0.10526315789473684);
  p = fma(p, z, 0.11764705882352941);
  p = fma(p, z, 0.13333333333333333);
  p = fma(p, z, 0.15384615384615385);
  p = fma(p, z, 0.18181818181818182);
  p = fma(p, z, 0.2222222222222222);
  p = fma(p, z, 0.2857142857142857);
  p = fma(p, z, 0.4);
  p = fma(p, z, 0.6666666666666666);
  const double lnm = fma(s * z, p, 2.0 * s);  // 2s + s z (2/3 + ...)
  const double E = (double)(e - 33);
  // ln 2 split so that E * ln2_hi is exact
  return fma(E, 0.6931471805601177, fma(E, -1.7239444525614835e-13, lnm));
}

// sqrt(v) for v in [2^-33, 64]: reciprocal square-root seed and two Newton
// steps (the second on the root itself).
__device__ __forceinline__ double sqrt_pos_f64(double v) {
  const double r0 = __builtin_amdgcn_rsq(v);
  double y = v * r0, h = 0.5 * r0;
  const double e = fma(-y, h, 0.5);
  y = fma(y, e, y);
  h = fma(h, e, h);
  return fma(fma(-y, y, v), h, y);
}

// 1/sqrt(v) for v >= 0 (0 for v = 0, so that v * inv_sqrt(v) = sqrt(v)):
// reciprocal square-root seed and two Newton steps.
__device__ __forceinline__ double inv_sqrt_f64(double v) {
  if (!(v > 0.0)) return 0.0;
  double r = __builtin_amdgcn_rsq(v);
  const double h = 0.5 * v;
  r = fma(r, fma(-h * r, r, 0.5), r);
  r = fma(r, fma(-h * r, r, 0.5), r);
  return r;
}

// sin(pi t) and cos(pi t) for t in [0, 2]: t = k/2 + y with k = rint(2t) and
// |y| <= 1/4 exactly; the Taylor series of sin(pi y) and cos(pi y) to the
// 17th and 16th power, then the quarter-turn k mod 4 rotates the pair.
__device__ __forceinline__ void sincospi_f64(double t, double& sn, double& cs) {
  const double k = rint(2.0 * t);
  const double y = fma(-0.5, k, t);  // exact
  const double w = y * y;
  double ps = 7.952054001475513e-07;
  ps = fma(ps, w, -2.1915353447830217e-05);
  ps = fma(ps, w, 0.00046630280576761255);
  ps = fma(ps, w, -0.0073704309457143504);
  ps = fma(ps, w, 0.08214588661112823);
  ps = fma(ps, w, -0.5992645293207921);
  ps = fma(ps, w, 2.5501640398773455);
  ps = fma(ps, w, -5.16771278004997);
  const double sp = fma(y * w, ps, 3.141592653589793 * y);
  double pc = 4.303069587032947e-06;
  pc = fma(pc, w, -0.0001046381049248457);
  pc = fma(pc, w, 0.0019295743094039231);
  pc = fma(pc, w, -0.02580689139001406);
  pc = fma(pc, w, 0.2353306303588932);
  pc = fma(pc, w, -1.3352627688545895);
  pc = fma(pc, w, 4.0587121264167685);
  pc = fma(pc, w, -4.934802200544679);
  const double cp = fma(w, pc, 1.0);
  const int q = (int)k & 3;
  const double a = (q & 1) ? cp : sp;  // sin of the rotated angle, up to sign
  const double b = (q & 1) ? sp : cp;  // cos of the rotated angle, up to sign
  sn = (q & 2) ? -a : a;
  cs = ((q + 1) & 2) ? -b : b;
}

// FP64 normals from the four words: u = (x + 1/2) 2^-32 in (0,1).
__device__ __forceinline__ void box_muller_f64(const uint32_t w[4], double G[3]) {
  const double s = 2.3283064365386963e-10;  // 2^-32
  const double r1 = sqrt_pos_f64(-2.0 * ln_uniform_f64(w[0]));
  const double r2 = sqrt_pos_f64(-2.0 * ln_uniform_f64(w[2]));
  const double t1 = (2.0 * (double)w[1] + 1.0) * s;  // 2 u1, exact
  const double t3 = (2.0 * (double)w[3] + 1.0) * s;
  double sn, cs, sn3, cs3;
  sincospi_f64(t1, sn, cs);
  sincospi_f64(t3, sn3, cs3);
  G[0] = r1 * cs;
  G[1] = r1 * sn;
  G[2] = r2 * cs3;
}

// The first normal only (the scalar noise of the projected model).
__device__ __forceinline__ double normal1_f64(const uint32_t w[4]) {
  const double r1 = sqrt_pos_f64(-2.0 * ln_uniform_f64(w[0]));
  double sn, cs;
  sincospi_f64((2.0 * (double)w[1] + 1.0) * 2.3283064365386963e-10, sn, cs);
  return r1 * cs;
}

// ln u for u = (x + 1/2) 2^-32 in FP32.  Far from 1 the float of x keeps 24
// significant bits at every magnitude (the tails keep full relative
// precision); within 2^-8 of 1, ln u = ln(1 - v) is summed as a series in the
// complement v = (~x + 1/2) 2^-32, which the float grid below 1 cannot resolve.
__device__ __forceinline__ float ln_uniform_f32(uint32_t x) {
  const float two_m32 = 2.3283064365386963e-10f;
  if (x >= 0xFF000000u) {
    const float v = ((float)(~x) + 0.5f) * two_m32;
    return -v * (1.0f + v * (0.5f + v * 0.33333334f));
  }
  const float u = ((float)x + 0.5f) * two_m32;
  return 0.6931471805599453f * __builtin_amdgcn_logf(u);  // ln 2 * log2 u
}

// FP32 normals from the same words; the hardware sine/cosine take their
// argument in turns, so sin(2 pi u) is one instruction.
__device__ __forceinline__ void box_muller_f32(const uint32_t w[4], float G[3]) {
  const float two_m32 = 2.3283064365386963e-10f;
  const float r1 = __builtin_sqrtf(-2.0f * ln_uniform_f32(w[0]));
  const float r2 = __builtin_sqrtf(-2.0f * ln_uniform_f32(w[2]));
  const float u1 = (float)w[1] * two_m32;
  const float u3 = (float)w[3] * two_m32;
  G[0] = r1 * __builtin_amdgcn_cosf(u1);
  G[1] = r1 * __builtin_amdgcn_sinf(u1);
  G[2] = r2 * __builtin_amdgcn_cosf(u3);
}

__device__ __forceinline__ float normal1_f32(const uint32_t w[4]) {
  const float r1 = __builtin_sqrtf(-2.0f * ln_uniform_f32(w[0]));
  return r1 * __builtin_amdgcn_cosf((float)w[1] * 2.3283064365386963e-10f);
}

// -------------------------------------------------------------------------
// Geometry.
// -------------------------------------------------------------------------
__device__ __forceinline__ double wrap_coord(double x, double L) {
  if (x < 0.0 || x >= L) {
    x = x - L * floor(x / L);
    if (x >= L) x = 0.0;
  }
  return x;
}

// d - L if d > L/2, d + L if d < -L/2, else d (selects, no branches: the
// lanes of a wave take different cases)
__device__ __forceinline__ double min_image(double d, double L, double halfL) {
  const double lo = d - L, hi = d + L;
  d = d > halfL ? lo : d;
  return d < -halfL ? hi : d;
}

// r^2 evaluated as (dx*dx + dy*dy) + dz*dz with no fused multiply-add, so the
// pair predicate r^2 < rc^2 is an exact function of the positions.
__device__ __forceinline__ double dist2(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  const double xx = dx * dx;
  const double yy = dy * dy;
  const double zz = dz * dz;
  return (xx + yy) + zz;
}

__device__ __forceinline__ int cell_coord(double x, double scale, int nc) {
  double c = floor(x * scale);
  c = (c >= 0.0) ? c : 0.0;  // also maps NaN to 0 so indices stay in range
  c = (c <= (double)(nc - 1)) ? c : (double)(nc - 1);
  return (int)c;
}

// Memory order of the cells (the particles are kept sorted by this key):
// blocks of oblk^3 cells in row-major block order, row-major cells inside a
// block, the blocks at the high faces cut to the box; oblk = 1 is the
// row-major order of the cells.  The map is a bijection onto
// [0, nc0 nc1 nc2), and cells that follow each other along x inside one
// block have consecutive keys.  Compact blocks keep more of a particle's
// neighbours in the particles stored next to it.
// c / oblk for a cell coordinate 0 <= c <= 10^6 (the host's limit on cells
// per axis) and a block edge of 1..8: (c + 1/2) / oblk from the FP32
// reciprocal in one fused multiply-add lies within 2^-2 / oblk of its exact
// value, whose distance from an integer is at least 1 / (2 oblk), so the
// truncation is the quotient (checked for every c < 2^21 on the host).  It
// replaces an integer division sequence in the list build's stencil setup.
__device__ __forceinline__ int block_of(int c, const Geo& g) {
  return (int)__builtin_fmaf((float)c, g.oblk_inv, 0.5f * g.oblk_inv);
}

__device__ __forceinline__ uint32_t cell_key(const Geo& g, int cx, int cy, int cz) {
  const int64_t n0 = g.nc[0], n1 = g.nc[1];
  const int B = g.oblk;
  if (B == 1) return (uint32_t)(cx + n0 * (cy + n1 * cz));
  const int bx = block_of(cx, g), by = block_of(cy, g), bz = block_of(cz, g);
  const int sx = min(B, g.nc[0] - bx * B), sy = min(B, g.nc[1] - by * B),
            sz = min(B, g.nc[2] - bz * B);
  const int lx = cx - bx * B, ly = cy - by * B, lz = cz - bz * B;
  return (uint32_t)(n0 * n1 * (bz * B) + n0 * sz * (by * B) + (int64_t)sy * sz * (bx * B) + lx +
                    sx * (ly + sy * lz));
}

// -------------------------------------------------------------------------
// Deterministic reductions: xor-butterfly inside a wave (every lane ends with
// the same bits), then waves combined in index order by one thread.
// -------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* smem /* NV * nwaves */) {
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) smem[k * nw + wid] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += smem[k * nw + w];
      v[k] = s;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Order-independent sums.  A value x (|x| < 2^31) is rounded once to the grid
// 2^-64 and held as a 128-bit two's-complement integer (hi:lo); integer
// addition is associative, so a sum of such values is the same bit pattern
// whatever the order, tiling or memory layout of its terms.
// ---------------------------------------------------------------------------
struct Fix {
  uint64_t lo;
  int64_t hi;
};

__device__ __forceinline__ Fix fix_zero() { return Fix{0ull, 0ll}; }

__device__ __forceinline__ Fix fix_add(Fix a, Fix b) {
  Fix r;
  r.lo = a.lo + b.lo;
  r.hi = a.hi + b.hi + (r.lo < a.lo ? 1ll : 0ll);
  return r;
}

// round(x * 2^64): x * 2^32 = h + f exactly with h = floor(x * 2^32) and
// f in [0, 1); the only rounding is that of f * 2^32 to an integer.
__device__ __forceinline__ Fix fix_of(double x) {
  const double y = x * 0x1p32;
  const double yh = floor(y);
  const int64_t h = (int64_t)yh;
  const uint64_t l = (uint64_t)rint((y - yh) * 0x1p32);
  Fix r;
  r.lo = ((uint64_t)h << 32);
  r.hi = h >> 32;
  return fix_add(r, Fix{l, 0ll});
}

__device__ __forceinline__ double fix_to_double(Fix a) {
  return (double)a.hi + (double)a.lo * 0x1p-64;
}

__device__ __forceinline__ Fix wave_sum_fix(Fix a) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    Fix b;
    b.lo = (uint64_t)__shfl_xor((long long)a.lo, off, kWave);
    b.hi = (int64_t)__shfl_xor((long long)a.hi, off, kWave);
    a = fix_add(a, b);
  }
  return a;
}

// Block-wide sums of NV fixed-point values; thread 0 holds the result.
template <int NV>
__device__ __forceinline__ void block_sum_fix(Fix (&v)[NV], Fix* smem /* NV * nwaves */) {
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum_fix(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) smem[k * nw + wid] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      Fix s = fix_zero();
      for (int w = 0; w < nw; ++w) s = fix_add(s, smem[k * nw + w]);
      v[k] = s;
    }
  }
  __syncthreads();
}

__device__ __forceinline__ bool status_set(const uint32_t* status) { return *status != 0u; }

}  // namespace dpde
