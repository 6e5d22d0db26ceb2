// Pair passes of one DPDE step over cell-sorted particles.
//
//   pass A  conservative forces at the new positions, neighbour list build,
//           second half-kick of velocity-Verlet (Sec. 3.1);
//   pass B  SER sweep 1: dp_ij and dp_i = sum_j dp_ij (eq. SER_p);
//   pass C  SER sweep 2: internal-energy reinjection
//           (eq. SER_eint_discretization), p <- p + dp, eps <- eps + d eps,
//           next 1/T_i.
//
// One lane per particle; each pair term is evaluated on both of its
// particles' lanes in the canonical orientation (lower identifier first) and
// negated on the higher one, so dp_ji = -dp_ij bit for bit and the particle
// sums are plain gathers: no atomics, fixed summation order.
//
// Sweep 2 needs the same dp_ij as sweep 1.  The paper regenerates the noise
// from (i, j, n) to avoid storing the increments; with HBM to spare, sweep 1
// here stores dp_ij per neighbour-list entry and sweep 2 reads it back, which
// removes the random-number generation and the pair geometry from sweep 2.
// The regenerating form is kept (Phys::regen) and gives identical bits.
#pragma once

#include "bin.h"
#include "eos.h"
#include "mlp.h"

namespace dpde {

constexpr int kPairBlockMax = 256;

enum : int { PREC_F64 = 0, PREC_F32 = 1 };

struct alignas(32) DP {
  double x, y, z, pad;
};

// Momentum after the conservative half-kick and the sweep-1 increment of one
// particle, packed so that sweep 2 gathers one line per neighbour.
// Per-particle results of SER sweep 1: dp_i = sum_j dp_ij, and
// h_i = (p_i + dp_i / 2) / m, so that the velocity combination of sweep 2,
// v_ij + (dp_i - dp_j)/(2m), is h_i - h_j (exactly antisymmetric).
struct alignas(32) Vec4 {
  double x, y, z, w;
};

// Neighbour list: k-major (entry k of particle i at k*n + i), so the lanes of
// a wave read and write consecutive words for a given k.
struct NList {
  uint32_t* idx;
  uint32_t* count;
  double *dex, *dey, *dez;  // dp_ij per entry (stored-increment form), same layout
  int64_t stride;           // n
};

// Up to two contiguous cell ranges along x for the stencil row (y, z).
struct Row {
  int a0, b0, a1, b1;  // inclusive cell x-ranges; a1 > b1 means "no second range"
};

__device__ __forceinline__ Row stencil_row(int cx, int nc, int periodic) {
  Row r;
  r.a1 = 1;
  r.b1 = 0;
  if (periodic) {
    if (cx == 0) { r.a0 = 0; r.b0 = 1; r.a1 = nc - 1; r.b1 = nc - 1; }
    else if (cx == nc - 1) { r.a0 = nc - 2; r.b0 = nc - 1; r.a1 = 0; r.b1 = 0; }
    else { r.a0 = cx - 1; r.b0 = cx + 1; }
  } else {
    r.a0 = cx > 0 ? cx - 1 : 0;
    r.b0 = cx < nc - 1 ? cx + 1 : nc - 1;
  }
  return r;
}

__device__ __forceinline__ bool wrap_cell(int& c, int nc, int periodic) {
  if (c < 0) {
    if (!periodic) return false;
    c += nc;
  } else if (c >= nc) {
    if (!periodic) return false;
    c -= nc;
  }
  return true;
}

// Separation q_i - q_j with the minimum image along periodic dimensions.
__device__ __forceinline__ void separation(const Geo& g, double xi, double yi, double zi,
                                           double xj, double yj, double zj, double& dx,
                                           double& dy, double& dz) {
  dx = xi - xj;
  dy = yi - yj;
  dz = zi - zj;
  if (g.periodic[0]) dx = min_image(dx, g.box[0], g.half_box[0]);
  if (g.periodic[1]) dy = min_image(dy, g.box[1], g.half_box[1]);
  if (g.periodic[2]) dz = min_image(dz, g.box[2], g.half_box[2]);
}

// A particle farther than the list reach from every periodic face sees all of
// its listed neighbours at their stored (wrapped) positions: the minimum
// image is then the identity.  Waves whose particles all qualify skip it.
__device__ __forceinline__ bool away_from_faces(const Geo& g, const Phys& P, double x, double y,
                                                double z) {
  const double q[3] = {x, y, z};
  bool ok = true;
#pragma unroll
  for (int d = 0; d < 3; ++d)
    if (g.periodic[d]) ok = ok && q[d] >= P.reach && q[d] <= g.box[d] - P.reach;
  return ok;
}

__device__ __forceinline__ void separation_mi(const Geo& g, bool mi, double xi, double yi,
                                              double zi, double xj, double yj, double zj,
                                              double& dx, double& dy, double& dz) {
  if (mi) {
    separation(g, xi, yi, zi, xj, yj, zj, dx, dy, dz);
  } else {
    dx = xi - xj;
    dy = yi - yj;
    dz = zi - zj;
  }
}

// ---------------------------------------------------------------------------
// Lane groups.  Every particle is served by kSub consecutive lanes of one
// wave: lane `sub` of the group takes the list entries sub, sub + kSub, ...,
// and partial sums meet in a fixed xor butterfly.  The butterfly adds the same
// two operands on both partner lanes (in swapped order, which addition does
// not see), so all lanes of a group end with the same, reproducible sum.
// Compaction into a list keeps the candidates' order: each trip the group
// ballots its predicates and a lane's slot is the count of set bits below it.
// ---------------------------------------------------------------------------
constexpr int kSub = 4;
constexpr uint32_t kSubMask = (1u << kSub) - 1u;
// The SER sweeps (passes B and C) use pairs of lanes: with ~12 neighbours
// their pair terms keep more lanes busy per trip, while the filters over the
// ~27 skin candidates (pass A, list build) are faster with four.
constexpr int kSubSer = 2;
constexpr int kListLds = 64;  // list entries per particle staged in LDS
constexpr int kBuildLds = 32;  // the same in the list build
constexpr int kUniqTile = 128;  // particles per tile (= block) of the unique-pair passes

// In the tile form a pair joining two particles of one tile (128 consecutive
// memory indices) is listed for one of them only: for the lower memory index
// when the two indices differ in parity, else for the higher one, so that
// about half of every particle's pairs inside its tile stay in its list
// whatever its place in the tile (the lanes of the passes stay evenly
// loaded).  Which side evaluates a pair changes no sum: every per-particle sum
// of the tile form is an exact fixed-point sum.
__device__ __forceinline__ bool tile_listed(uint32_t i, uint32_t j) {
  if ((i ^ j) >= (uint32_t)kUniqTile) return true;  // different tiles: both lists
  return ((i ^ j) & 1u) ? (i < j) : (i > j);
}

// Exclusive prefix of v over the wave and the wave total.
__device__ __forceinline__ uint32_t wave_prefix(uint32_t v, uint32_t& total) {
  const int lane = threadIdx.x % kWave;
  uint32_t incl = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t up = (uint32_t)__shfl_up((int)incl, off, kWave);
    if (lane >= off) incl += up;
  }
  total = (uint32_t)__shfl((int)incl, kWave - 1, kWave);
  return incl - v;
}

struct Lanes {
  int64_t i;     // particle
  int sub;       // lane within the group
  int pib;       // group within the block
  int ppb;       // groups per block
  int shift;     // position of the group's bits in a wave ballot
};

template <int KS = kSub>
__device__ __forceinline__ Lanes lanes() {
  Lanes L;
  const int64_t t = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  L.i = t / KS;
  L.sub = threadIdx.x % KS;
  L.pib = threadIdx.x / KS;
  L.ppb = blockDim.x / KS;
  L.shift = (threadIdx.x % kWave) & ~(KS - 1);
  return L;
}

template <int KS = kSub>
__device__ __forceinline__ double group_sum(double x) {
#pragma unroll
  for (int off = 1; off < KS; off <<= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

// Group bits of a wave ballot.
__device__ __forceinline__ uint32_t group_ballot(const Lanes& L, bool pred) {
  return (uint32_t)(__ballot(pred) >> L.shift) & kSubMask;
}

// Visit the 27-cell stencil.  Its cells come as runs of consecutive memory
// (three cells of an x-row in row-major order; one run per cell block an
// x-row crosses in blocked order; a periodic wrap splits a row), which the
// group first lists in LDS (`runs`: the runs' first indices, then their
// cumulative ends with the run's periodic image in the top bits); the
// group's lanes then take the concatenated candidates four at a time (lane
// sub takes position F + sub), so a trip is cut short only at the end of the
// stencil, not at the end of every run.  A run reached across a periodic face
// holds images one box length away: its candidates are compared after that
// shift (d - s with s = +-L), which for every candidate within the list
// radius is the minimum image itself, with the same two roundings.
// `sink(take, j, id_j)` is called on every trip, `take` being r^2 < thr2 and
// j != i; the trips are uniform across the group, so `sink` may ballot.
constexpr int kRunsMax = 28;  // runs per stencil: 9 rows x at most 3 pieces
constexpr int kRunEndBits = 26;  // cumulative end; above it 2 bits per axis: 1 = +L, 2 = -L

template <bool MI, typename Sink>
__device__ __forceinline__ bool scan_candidates(const Lanes& L, const Geo& g,
                                                const uint32_t* __restrict__ start,
                                                const QIdF* __restrict__ qid, float xi, float yi,
                                                float zi, int cx, int cy, int cz, float thr2,
                                                uint32_t* runs, Sink&& sink) {
  const float bx = (float)g.box[0], by = (float)g.box[1], bz = (float)g.box[2];
  // the runs, in stencil order (uniform across the group; lane 0 records)
  uint32_t nr = 0, tot = 0;
  bool whole = true;  // false: the stencil holds more candidates than the run ends can count
  constexpr uint32_t kEndMask = (1u << kRunEndBits) - 1u;
  auto add = [&](uint32_t jb, uint32_t je, uint32_t image) {
    if (je > jb && je - jb > kEndMask - tot) whole = false;
    if (je > jb && whole) {
      tot += je - jb;
      if (L.sub == 0) {
        runs[nr] = jb;
        runs[kRunsMax + nr] = tot | (image << kRunEndBits);
      }
      ++nr;
    }
  };
  // the image code of a neighbour cell index before wrapping: +L from above,
  // -L from below (2 bits)
  auto code = [](int c, int nc) -> uint32_t { return c >= nc ? 1u : (c < 0 ? 2u : 0u); };
  const Row row = stencil_row(cx, g.nc[0], g.periodic[0]);
  const int B = g.oblk;
  // the x image of the second range of a periodic row: the cell left of
  // cx = 0 or right of cx = nc - 1
  const uint32_t cx1 = cx == 0 ? 2u : 1u;
  for (int dz = -1; dz <= 1; ++dz) {
    int z = cz + dz;
    const uint32_t iz = code(z, g.nc[2]) << 4;
    if (!wrap_cell(z, g.nc[2], g.periodic[2])) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      int y = cy + dy;
      const uint32_t iyz = iz | (code(y, g.nc[1]) << 2);
      if (!wrap_cell(y, g.nc[1], g.periodic[1])) continue;
      if (B == 1) {  // row-major cells: each x range is one run of memory
        const int64_t base = g.cell_base + (int64_t)g.nc[0] * (y + (int64_t)g.nc[1] * z);
        add(start[base + row.a0], start[base + row.b0 + 1], iyz);
        if (row.a1 <= row.b1) add(start[base + row.a1], start[base + row.b1 + 1], iyz | cx1);
      } else {
        // blocked order: an x range is one run per cell block it crosses
        auto xrun = [&](int a, int b, uint32_t image) {
          for (int x = a; x <= b;) {
            const int e = min(b, block_of(x, g) * B + B - 1);
            const int64_t k0 = g.cell_base + cell_key(g, x, y, z);
            add(start[k0], start[k0 + (e - x) + 1], image);
            x = e + 1;
          }
        };
        xrun(row.a0, row.b0, iyz);
        if (row.a1 <= row.b1) xrun(row.a1, row.b1, iyz | cx1);
      }
    }
  }
  // the group's lanes read what lane 0 wrote (one wave: a fence suffices)
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  auto shift = [](uint32_t c2, float l) { return c2 == 1u ? l : (c2 == 2u ? -l : 0.0f); };
  // lane-local cursor: run r covers concatenated positions [prev, end) and
  // holds images shifted by (sx, sy, sz)
  uint32_t r = 0, prev = 0, word = nr ? runs[kRunsMax] : 0u;
  uint32_t end = word & kEndMask;
  float sx = 0.0f, sy = 0.0f, sz = 0.0f;
  auto image = [&]() {
    if constexpr (MI) {
      const uint32_t c = word >> kRunEndBits;
      sx = shift(c & 3u, bx);
      sy = shift((c >> 2) & 3u, by);
      sz = shift(c >> 4, bz);
    }
  };
  image();
  for (uint32_t F = 0; F < tot; F += kSub) {
    const uint32_t f = F + L.sub;
    bool take = false;
    uint32_t j = 0, idj = 0;
    if (f < tot) {
      if (f >= end) {
        do {
          prev = end;
          ++r;
          word = runs[kRunsMax + r];
          end = word & kEndMask;
        } while (f >= end);
        image();
      }
      j = runs[r] + (f - prev);
      const QIdF c = qid[j];
      float dx = xi - c.x, dy = yi - c.y, dz = zi - c.z;
      if constexpr (MI) {
        dx -= sx;
        dy -= sy;
        dz -= sz;
      }
      idj = c.id;
      take = (dx * dx + dy * dy) + dz * dz < thr2 && j != (uint32_t)L.i;
    }
    sink(take, j, idj);
  }
  return whole;
}


// ---------------------------------------------------------------------------
__device__ __forceinline__ bool interior_dim(int c, int nc, int periodic) {
  // cells c-1..c+1 exist without wrapping
  return !periodic || (c >= 1 && c <= nc - 2);
}

// Neighbour lists with a skin.  On a build step every particle collects the
// particles within rs = rc + skin through the 27-cell stencil (scan_candidates),
// and the list is sorted by neighbour identifier.  Every step then keeps the
// entries with r < rc, in list order: the pair set is exactly the stencil's,
// and every per-particle sum below runs in identifier order, so the
// trajectory does not depend on memory order, skin width or build schedule.
// A build is due when some particle has moved more than skin/2 since the last
// one (then no pair within rc can be missing from the lists).
// ---------------------------------------------------------------------------
struct SkinList {
  uint32_t* idx;    // k-major, capacity cap per particle
  uint32_t* count;
  int64_t stride;   // n
  int32_t cap;
  int32_t pad;
};

// With `uniq` (the tile form) the list keeps only the pairs tile_listed
// assigns to this particle, holds memory indices, and is not sorted: the
// passes that read it add their pair terms in fixed point, in any order.
// s holds the records the reorder has just written in cell order (its
// candidates come from qid); the group's first lane also returns its
// particle's record and internal energy to the working buffer `work`.
template <bool BATCH>
__global__ __launch_bounds__(kPairBlockMax) void k_build_skin(
    PState s, PState work, const QIdF* __restrict__ qid, const uint32_t* __restrict__ start,
    int64_t n, const Geo* __restrict__ geo, double rs, double box_max, SkinList sl,
    const BuildCtl* ctl, double half_skin2, int uniq, uint32_t* status) {
  __shared__ uint32_t lst[kBuildLds * (kPairBlockMax / kSub)];
  __shared__ uint32_t runs_s[2 * kRunsMax * (kPairBlockMax / kSub)];
  if (status_set(status) || !rebuild_now(ctl, half_skin2)) return;  // uniform
  const Lanes L = lanes();
  if (L.i >= n) return;  // uniform in the group
  uint32_t* runs = runs_s + 2 * kRunsMax * L.pib;
  const int64_t i = L.i;
  const Rec* __restrict__ R = s.r;
  if (L.sub == 0) {
    work.r[i] = R[i];
    work.eps[i] = s.eps[i];
  }
  const double xi = R[i].qx, yi = R[i].qy, zi = R[i].qz;
  const Geo& g = geo[BATCH ? R[i].rep : 0u];
  // FP32 test radius: rs plus a bound on the rounding of the FP32 distance
  // (conversions of coordinates up to Q = max(|q|, box), their difference,
  // the minimum image and the squared sum stay below 8 2^-24 (Q + rs); twice
  // that is added), rounded up
  const double Q = fmax(__longlong_as_double((long long)ctl->qmax_bits), box_max);
  const double thr = rs + 16.0 * 0x1p-24 * (Q + rs);
  float thr2 = (float)(thr * thr);
  if ((double)thr2 < thr * thr) thr2 = nextafterf(thr2, INFINITY);
  const QIdF own = qid[i];
  const int cx = cell_coord(xi, g.scale[0], g.nc[0]);
  const int cy = cell_coord(yi, g.scale[1], g.nc[1]);
  const int cz = cell_coord(zi, g.scale[2], g.nc[2]);
  uint32_t nn = 0;
  const uint32_t cap = (uint32_t)sl.cap;
  // the list holds identifier rows (first + id) until k_sort_skin has
  // ordered them and turned them into memory indices
  const uint32_t first = (uint32_t)g.first;
  auto sink = [&](bool take, uint32_t j, uint32_t idj) {
    if (uniq) take = take && tile_listed((uint32_t)i, j);
    const uint32_t bits = group_ballot(L, take);
    if (take) {
      const uint32_t pos = nn + __popc(bits & ((1u << L.sub) - 1u));
      const uint32_t row = uniq ? j : first + idj;
      if (pos < (uint32_t)kBuildLds) lst[pos * L.ppb + L.pib] = row;
      else if (pos < cap) sl.idx[(int64_t)pos * sl.stride + i] = row;
    }
    nn += __popc(bits);
  };
  // waves whose particles all sit away from the periodic faces meet no
  // image across them
  const bool interior = interior_dim(cx, g.nc[0], g.periodic[0]) &&
                        interior_dim(cy, g.nc[1], g.periodic[1]) &&
                        interior_dim(cz, g.nc[2], g.periodic[2]);
  const bool whole =
      __all(interior)
          ? scan_candidates<false>(L, g, start, qid, own.x, own.y, own.z, cx, cy, cz, thr2, runs,
                                   sink)
          : scan_candidates<true>(L, g, start, qid, own.x, own.y, own.z, cx, cy, cz, thr2, runs,
                                  sink);
  // a stencil too full to count is a list overflow
  if (!whole && L.sub == 0) atomicOr(status, ST_OVERFLOW);
  if (nn > cap) {
    if (L.sub == 0) atomicOr(status, ST_OVERFLOW);
    nn = cap;
  }
  const uint32_t staged = nn < (uint32_t)kBuildLds ? nn : (uint32_t)kBuildLds;
  for (uint32_t k = L.sub; k < staged; k += kSub)
    sl.idx[(int64_t)k * sl.stride + i] = lst[k * L.ppb + L.pib];
  if (L.sub == 0) sl.count[i] = nn;
}

// Sort each skin list by neighbour identifier and replace the identifier
// rows by memory indices (slot[row], written by the reorder).  One list per
// lane, held in registers padded with all-ones and sorted by a bitonic
// network of 32, 64 or (for long lists, MAXW = 128) 128 words (the wave's
// longest list picks the width; rows are unique, so the order is total).
// Longer lists are insertion-sorted in place in global memory.
template <int N>
__device__ __forceinline__ void bitonic_sort(uint32_t (&v)[N]) {
#pragma unroll
  for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int e = 0; e < N; ++e) {
        const int l = e ^ j;
        if (l > e) {
          const uint32_t x = v[e], y = v[l];
          const bool up = (e & k) == 0;
          v[e] = up ? min(x, y) : max(x, y);
          v[l] = up ? max(x, y) : min(x, y);
        }
      }
    }
  }
}

template <int N>
__device__ __forceinline__ void sort_list_regs(const SkinList& sl, const uint32_t* __restrict__ slot,
                                               int64_t i, uint32_t nn) {
  uint32_t v[N];
  const int64_t st = sl.stride;
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = (uint32_t)k < nn ? sl.idx[k * st + i] : 0xFFFFFFFFu;
  bitonic_sort<N>(v);
#pragma unroll
  for (int k = 0; k < N; ++k)
    if ((uint32_t)k < nn) sl.idx[k * st + i] = slot[v[k]];
}

template <int MAXW>
__global__ __launch_bounds__(256) void k_sort_skin(int64_t n, SkinList sl,
                                                   const uint32_t* __restrict__ slot,
                                                   const BuildCtl* ctl, double half_skin2,
                                                   const uint32_t* status) {
  if (status_set(status) || !rebuild_now(ctl, half_skin2)) return;  // uniform
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nn = i < n ? sl.count[i] : 0u;
  uint32_t wmax = nn;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1)
    wmax = max(wmax, (uint32_t)__shfl_xor((int)wmax, off, kWave));
  if (i >= n || nn == 0) return;
  if (wmax <= 32u) {
    sort_list_regs<32>(sl, slot, i, nn);
  } else if (nn <= 64u && (MAXW == 64 || wmax <= 64u)) {
    sort_list_regs<64>(sl, slot, i, nn);
  } else if (MAXW >= 128 && nn <= 128u) {
    sort_list_regs<MAXW>(sl, slot, i, nn);
  } else {
    const int64_t st = sl.stride;
    for (uint32_t m = 1; m < nn; ++m) {
      const uint32_t x = sl.idx[m * st + i];
      uint32_t q = m;
      while (q > 0) {
        const uint32_t y = sl.idx[(q - 1) * st + i];
        if (y <= x) break;
        sl.idx[q * st + i] = y;
        --q;
      }
      sl.idx[q * st + i] = x;
    }
    for (uint32_t m = 0; m < nn; ++m) sl.idx[m * st + i] = slot[sl.idx[m * st + i]];
  }
}

// Pass A: neighbour list of the step (skin entries with r < rc, in identifier
// order, staged in LDS and written out coalesced), forces
// F_i = -sum_j v'(r_ij) d_ij / r_ij, U_i = 1/2 sum_j v(r_ij) and the Laplacian
// share L_i = sum_j (v'' + 2 v'/r) (eq. Tcon); mode 1 also applies
// p += dt/2 F (end of velocity-Verlet).  v is the soft potential
// (a rc/2)(1 - r/rc)^2 or the splined LJ of eq. Ep.
template <bool BATCH, int PREC>
__global__ __launch_bounds__(kPairBlockMax) void k_pass_a(
    PState s, int64_t n, const Geo* __restrict__ geo, Phys P, int mode,
    double* __restrict__ Fx, double* __restrict__ Fy, double* __restrict__ Fz,
    double* __restrict__ Ui, double* __restrict__ Li, SkinList sl, NList nl, uint32_t* status) {
  __shared__ uint32_t lst[kListLds * (kPairBlockMax / kSub)];
  const Lanes L = lanes();
  if (L.i >= n) return;  // uniform in the group
  if (status_set(status)) return;
  const int64_t i = L.i;
  const Rec* __restrict__ R = s.r;
  const double xi = R[i].qx, yi = R[i].qy, zi = R[i].qz;
  const GeoRef<BATCH> g = geo[BATCH ? R[i].rep : 0u];
  const uint32_t ns = sl.count[i];
  const uint32_t cap = (uint32_t)P.cap;
  const bool mi = !__all(away_from_faces(g, P, xi, yi, zi));  // uniform in the wave
  uint32_t nn = 0;
  double fx = 0.0, fy = 0.0, fz = 0.0, u = 0.0, lap = 0.0;
  const float inv_rc_f = (float)P.inv_rc, a_f = (float)P.a;
  uint32_t jn = (uint32_t)L.sub < ns ? sl.idx[(int64_t)L.sub * sl.stride + i] : 0u;
  double qnx = 0.0, qny = 0.0, qnz = 0.0;
  if ((uint32_t)L.sub < ns) {
    qnx = R[jn].qx;
    qny = R[jn].qy;
    qnz = R[jn].qz;
  }
  for (uint32_t base = 0; base < ns; base += kSub) {
    const uint32_t k = base + L.sub;
    const uint32_t j = jn;
    const double qjx = qnx, qjy = qny, qjz = qnz;
    if (k + kSub < ns) {
      jn = sl.idx[(int64_t)(k + kSub) * sl.stride + i];
      qnx = R[jn].qx;
      qny = R[jn].qy;
      qnz = R[jn].qz;
    }
    bool take = false;
    double dx = 0.0, dy = 0.0, dz = 0.0, r2 = 0.0;
    if (k < ns) {
      separation_mi(g, mi, xi, yi, zi, qjx, qjy, qjz, dx, dy, dz);
      r2 = dist2(dx, dy, dz);
      take = r2 < P.rc2;
    }
    const uint32_t bits = group_ballot(L, take);
    const uint32_t c = __popc(bits);
    if (take) {
      const uint32_t pos = nn + __popc(bits & ((1u << L.sub) - 1u));
      if (pos < (uint32_t)kListLds) lst[pos * L.ppb + L.pib] = j;
      else if (pos < cap) nl.idx[(int64_t)pos * nl.stride + i] = j;
    }
    // the pair at list position p is summed by lane p mod kSub (as in passes
    // B and C), whichever lane tested it: lane sub owns rank r of this trip
    const uint32_t r = (uint32_t)(L.sub - (int)nn) & (uint32_t)(kSub - 1);
    uint32_t b = bits;
    for (uint32_t q = 0; q < r; ++q) b &= b - 1u;
    const int src = L.shift + (b ? __ffs(b) - 1 : 0);
    const double ox = __shfl(dx, src, kWave), oy = __shfl(dy, src, kWave);
    const double oz = __shfl(dz, src, kWave), orr = __shfl(r2, src, kWave);
    if (r < c) {
      if constexpr (PREC == PREC_F64) {
        const double ir = inv_sqrt_f64(orr);  // 0 at r = 0
        const double rr = orr * ir;
        double f;
        if (P.potential == 0) {
          const double w = 1.0 - rr * P.inv_rc;
          u += P.half_a_rc * w * w;
          f = P.a * w * ir;  // -v'(r)/r
          lap += ir > 0.0 ? P.a * P.inv_rc - 2.0 * P.a * w * ir : 0.0;
        } else {
          const double ir2 = ir * ir;
          const double s2 = P.r_lj2 * ir2;
          const double s6 = s2 * s2 * s2, s12 = s6 * s6;
          u += P.lj4e * (s12 - s6) - P.lj_vc - P.lj_dvc * (rr - P.rc);
          const double dv = -6.0 * P.lj4e * (2.0 * s12 - s6) * ir - P.lj_dvc;
          f = -dv * ir;
          lap += P.lj4e * (156.0 * s12 - 42.0 * s6) * ir2 + 2.0 * dv * ir;
        }
        fx += f * ox;
        fy += f * oy;
        fz += f * oz;
      } else {
        const float rr = __builtin_sqrtf((float)orr);
        const float ir = rr > 0.0f ? 1.0f / rr : 0.0f;
        float f;
        if (P.potential == 0) {
          const float w = 1.0f - rr * inv_rc_f;
          u += (double)((float)P.half_a_rc * w * w);
          f = a_f * w * ir;
          lap += (double)(rr > 0.0f ? a_f * inv_rc_f - 2.0f * a_f * w * ir : 0.0f);
        } else {
          const float ir2 = ir * ir;
          const float s2 = (float)P.r_lj2 * ir2;
          const float s6 = s2 * s2 * s2, s12 = s6 * s6;
          const float e4 = (float)P.lj4e;
          u += (double)(e4 * (s12 - s6) - (float)P.lj_vc - (float)P.lj_dvc * (rr - (float)P.rc));
          const float dv = -6.0f * e4 * (2.0f * s12 - s6) * ir - (float)P.lj_dvc;
          f = -dv * ir;
          lap += (double)(e4 * (156.0f * s12 - 42.0f * s6) * ir2 + 2.0f * dv * ir);
        }
        fx += (double)(f * (float)ox);
        fy += (double)(f * (float)oy);
        fz += (double)(f * (float)oz);
      }
    }
    nn += c;
  }
  fx = group_sum(fx);
  fy = group_sum(fy);
  fz = group_sum(fz);
  u = group_sum(u);
  lap = group_sum(lap);
  if (nn > cap) {
    if (L.sub == 0) atomicOr(status, ST_OVERFLOW);
    nn = cap;
  }
  const uint32_t staged = nn < (uint32_t)kListLds ? nn : (uint32_t)kListLds;
  for (uint32_t k = L.sub; k < staged; k += kSub)
    nl.idx[(int64_t)k * nl.stride + i] = lst[k * L.ppb + L.pib];
  if (L.sub == 0) {
    nl.count[i] = nn;
    Fx[i] = fx;
    Fy[i] = fy;
    Fz[i] = fz;
    Ui[i] = 0.5 * u;
    Li[i] = lap;
    if (mode) {
      Rec* W = s.r;
      W[i].px = W[i].px + P.half_dt * fx;
      W[i].py = W[i].py + P.half_dt * fy;
      W[i].pz = W[i].pz + P.half_dt * fz;
    }
  }
}

// ---------------------------------------------------------------------------
// The SER momentum increment of one pair as seen by particle i (eq. SER_p):
//   dp_ij = -gamma_ij chi v_ij dt + sigma sqrt(chi) G_ij sqrt(dt)
// with chi = w^2, w = 1 - r/rc, gamma_ij = (gamma kT/2)(1/T_i + 1/T_j) and
// G_ij = +G(lo,hi) for i = lo, -G(lo,hi) for i = hi.  Every factor is either
// symmetric in (i,j) or flips sign exactly, so the result for (j,i) is the
// exact negative.
// ---------------------------------------------------------------------------
struct PairOut {
  double dp[3];
  double gdotv;  // noise . velocity term of the SEM energy update
  double v2;     // squared velocity term of the SEM energy update
  double chi;
  double w;
  double gij;
};

// Model 1 (the original DPDE model, Sec. 2.1): friction and noise along
// e_ij = d_ij / r with one scalar normal xi_ij = xi_ji per pair,
//   dp_ij = (-gamma_ij chi (e_ij . v_ij) dt + sigma w xi_ij sqrt(dt)) e_ij,
// antisymmetric through e_ji = -e_ij; a coincident pair does not interact.
template <int PREC, int MODEL>
__device__ __forceinline__ void ser_pair(const Phys& P, const Geo& g, double dx, double dy,
                                         double dz, double r2, double vx, double vy, double vz,
                                         double invT_sum, uint32_t idi, uint32_t idj,
                                         uint64_t step, PairOut& o) {
  const bool i_lo = idi < idj;
  uint32_t wd[4];
  pair_words(g, i_lo ? idi : idj, i_lo ? idj : idi, step, wd);
  if constexpr (PREC == PREC_F64) {
    const double ir = inv_sqrt_f64(r2);
    const double r = r2 * ir;
    double w = 1.0 - r * P.inv_rc;
    const double gij = P.gkT_half * invT_sum;
    if constexpr (MODEL == 1) {
      if (!(r2 > 0.0)) w = 0.0;
      const double chi = w * w;
      const double ex = dx * ir, ey = dy * ir, ez = dz * ir;
      const double ev = ex * vx + ey * vy + ez * vz;
      const double xi = normal1_f64(wd);
      const double mag = -gij * chi * ev * P.dt + P.sigma * w * xi * P.sqrt_dt;
      o.dp[0] = mag * ex;
      o.dp[1] = mag * ey;
      o.dp[2] = mag * ez;
      o.gdotv = ev * xi;
      o.v2 = ev * ev;
      o.chi = chi;
      o.w = w;
      o.gij = gij;
      return;
    }
    const double chi = w * w;
    double G[3];
    box_muller_f64(wd, G);
    const double c1 = -gij * chi * P.dt;
    const double c2 = (i_lo ? P.sigma : -P.sigma) * w * P.sqrt_dt;
    o.dp[0] = c1 * vx + c2 * G[0];
    o.dp[1] = c1 * vy + c2 * G[1];
    o.dp[2] = c1 * vz + c2 * G[2];
    o.gdotv = (i_lo ? 1.0 : -1.0) * (G[0] * vx + G[1] * vy + G[2] * vz);
    o.v2 = vx * vx + vy * vy + vz * vz;
    o.chi = chi;
    o.w = w;
    o.gij = gij;
  } else {
    const float r = __builtin_sqrtf((float)r2);
    float w = 1.0f - r * (float)P.inv_rc;
    const float gij = (float)(P.gkT_half * invT_sum);
    const float v0 = (float)vx, v1 = (float)vy, v2 = (float)vz;
    if constexpr (MODEL == 1) {
      if (!(r > 0.0f)) w = 0.0f;
      const float chi = w * w;
      const float ir = r > 0.0f ? 1.0f / r : 0.0f;
      const float ex = (float)dx * ir, ey = (float)dy * ir, ez = (float)dz * ir;
      const float ev = ex * v0 + ey * v1 + ez * v2;
      const float xi = normal1_f32(wd);
      const float mag = -gij * chi * ev * (float)P.dt + (float)P.sigma * w * xi * (float)P.sqrt_dt;
      o.dp[0] = (double)(mag * ex);
      o.dp[1] = (double)(mag * ey);
      o.dp[2] = (double)(mag * ez);
      o.gdotv = (double)(ev * xi);
      o.v2 = (double)(ev * ev);
      o.chi = (double)chi;
      o.w = (double)w;
      o.gij = (double)gij;
      return;
    }
    const float chi = w * w;
    float G[3];
    box_muller_f32(wd, G);
    const float c1 = -gij * chi * (float)P.dt;
    const float c2 = (i_lo ? (float)P.sigma : -(float)P.sigma) * w * (float)P.sqrt_dt;
    o.dp[0] = (double)(c1 * v0 + c2 * G[0]);
    o.dp[1] = (double)(c1 * v1 + c2 * G[1]);
    o.dp[2] = (double)(c1 * v2 + c2 * G[2]);
    o.gdotv = (double)((i_lo ? 1.0f : -1.0f) * (G[0] * v0 + G[1] * v1 + G[2] * v2));
    o.v2 = vx * vx + vy * vy + vz * vz;
    o.chi = (double)chi;
    o.w = (double)w;
    o.gij = (double)gij;
  }
}

// dp_ij of neighbour j seen from the record of particle i.
template <int PREC, int MODEL>
__device__ __forceinline__ void pair_from_records(const Phys& P, const Geo& g, bool mi,
                                                  const Rec& a, const Rec& b, uint64_t step,
                                                  double& vx, double& vy, double& vz,
                                                  PairOut& o) {
  double dx, dy, dz;
  separation_mi(g, mi, a.qx, a.qy, a.qz, b.qx, b.qy, b.qz, dx, dy, dz);
  const double r2 = dist2(dx, dy, dz);
  vx = a.px * P.inv_mass - b.px * P.inv_mass;
  vy = a.py * P.inv_mass - b.py * P.inv_mass;
  vz = a.pz * P.inv_mass - b.pz * P.inv_mass;
  ser_pair<PREC, MODEL>(P, g, dx, dy, dz, r2, vx, vy, vz, a.invT + b.invT, a.id, b.id, step, o);
}

// Stored increments dp_ij: FP64, or FP32 for the FP32 pair terms, whose
// increments are FP32 values to begin with (exact either way).  They are
// written once and read once, so both go non-temporal: the stream does not
// evict the neighbour data the gathers of both sweeps reuse from L2.
template <int PREC>
__device__ __forceinline__ void store_dp(const NList& nl, int64_t e, double x, double y, double z) {
  if constexpr (PREC == PREC_F32) {
    __builtin_nontemporal_store((float)x, reinterpret_cast<float*>(nl.dex) + e);
    __builtin_nontemporal_store((float)y, reinterpret_cast<float*>(nl.dey) + e);
    __builtin_nontemporal_store((float)z, reinterpret_cast<float*>(nl.dez) + e);
  } else {
    __builtin_nontemporal_store(x, nl.dex + e);
    __builtin_nontemporal_store(y, nl.dey + e);
    __builtin_nontemporal_store(z, nl.dez + e);
  }
}

template <int PREC>
__device__ __forceinline__ void load_dp(const NList& nl, int64_t e, double& x, double& y,
                                        double& z) {
  if constexpr (PREC == PREC_F32) {
    x = (double)__builtin_nontemporal_load(reinterpret_cast<const float*>(nl.dex) + e);
    y = (double)__builtin_nontemporal_load(reinterpret_cast<const float*>(nl.dey) + e);
    z = (double)__builtin_nontemporal_load(reinterpret_cast<const float*>(nl.dez) + e);
  } else {
    x = __builtin_nontemporal_load(nl.dex + e);
    y = __builtin_nontemporal_load(nl.dey + e);
    z = __builtin_nontemporal_load(nl.dez + e);
  }
}

// h_i = (p_i + dp_i/2)/m packed in 24 bytes (gathered by sweep 2)
struct H3 {
  double x, y, z;
};

// ---------------------------------------------------------------------------
// Pass B (SER sweep 1, and the whole SEM update of eq. SEM_fd).
// ---------------------------------------------------------------------------
template <bool BATCH, int PREC, int SCHEME, int MODEL>
__global__ __launch_bounds__(kPairBlockMax) void k_pass_b(
    PState s, NList nl, int64_t n, const Geo* __restrict__ geo, Phys P,
    const uint64_t* __restrict__ d_step, Vec4* __restrict__ dpi, H3* __restrict__ hv,
    double* __restrict__ deps, int store, const uint32_t* __restrict__ dom, uint32_t* status) {
  const Lanes L = lanes<kSubSer>();
  if (L.i >= n) return;  // uniform in the group
  if (status_set(status)) return;
  const int64_t i = L.i;
  const uint64_t step = *d_step;
  const Rec* __restrict__ R = s.r;
  const Rec a = R[i];
  const GeoRef<BATCH> g = geo[BATCH ? a.rep : 0u];
  const bool mi = !__all(away_from_faces(g, P, a.qx, a.qy, a.qz));  // uniform in the wave
  const uint32_t nn = nl.count[i];
  const int64_t st = nl.stride;
  // Hybrid: pairs inside one domain were integrated by SSA; their entries
  // carry a zero increment here
  const uint32_t dom_i = dom ? dom[i] : 0u;
  double ax = 0.0, ay = 0.0, az = 0.0, de = 0.0;
  // no software pipeline: the registers a prefetched record would hold buy
  // one more wave per SIMD, which hides the gather latency better
  for (uint32_t k = L.sub; k < nn; k += kSubSer) {
    const int64_t e = (int64_t)k * st + i;
    const uint32_t j = nl.idx[e];
    const Rec b = R[j];
    if (dom && dom[j] == dom_i) {
      if (store) store_dp<PREC>(nl, e, 0.0, 0.0, 0.0);
      continue;
    }
    double vx, vy, vz;
    PairOut o;
    pair_from_records<PREC, MODEL>(P, g, mi, a, b, step, vx, vy, vz, o);
    ax += o.dp[0];
    ay += o.dp[1];
    az += o.dp[2];
    if (store) store_dp<PREC>(nl, e, o.dp[0], o.dp[1], o.dp[2]);
    if constexpr (SCHEME == 1) {
      de += 0.5 * (o.gij * o.v2 - P.dsigma2_m) * o.chi * P.dt -
            0.5 * P.sigma * o.w * o.gdotv * P.sqrt_dt;
    }
  }
  ax = group_sum<kSubSer>(ax);
  ay = group_sum<kSubSer>(ay);
  az = group_sum<kSubSer>(az);
  if constexpr (SCHEME == 1) de = group_sum<kSubSer>(de);
  if (L.sub == 0) {
    dpi[i] = Vec4{ax, ay, az, 0.0};
    hv[i] = H3{fma(ax, P.inv_2m, a.px * P.inv_mass), fma(ay, P.inv_2m, a.py * P.inv_mass),
                 fma(az, P.inv_2m, a.pz * P.inv_mass)};
    if constexpr (SCHEME == 1) deps[i] = de;
  }
}

// ---------------------------------------------------------------------------
// The SER sweeps with each pair inside a tile evaluated once.
//
// Tiles are 128 consecutive particles of the cell order (one block of the
// sweeps, two lanes per particle).  With cells of side rc + skin about half
// of all pairs join two particles of one tile.  Pass A leaves such a pair in
// the list of one of its particles only, so the sweeps evaluate it once:
// that particle adds the pair term to its own sum and, with an LDS atomic,
// to the partner's (negated in sweep 1, as dp_ji = -dp_ij exactly; unchanged
// in sweep 2, as the reinjection term is symmetric).  A pair joining two
// tiles stays in both lists and is evaluated for each particle, as before.
//
// The per-particle sums are exact integer sums of the terms rounded once to
// the grid 2^-46 (sums of 64-bit integers do not depend on the order of their
// terms).  A particle's sum is therefore the same bits whichever lane, wave
// or tile contributes each term, so trajectories still do not depend on the
// memory order, the neighbour-list skin, the rebuild schedule or the
// batching.  The conversion is exact-range for |term| < 32 (a momentum or
// energy increment of one pair in one step); a larger term stops the step
// with DPDE_ERANGE.
// ---------------------------------------------------------------------------
// Fixed-point pair sums.  x 2^46 is exact, and adding M = 1.5 2^52 rounds it
// to an integer held in the low mantissa bits while |x| < 32: the bit
// pattern of x 2^46 + M minus that of M is round(x 2^46).  A lane adds the
// raw bit patterns and subtracts count * M once at the end.  The range is
// tracked as the largest high word of |x| (a NaN or infinity exceeds it too).
constexpr long long kFixMagicBits = 0x4338000000000000ll;  // bits of 1.5 2^52
constexpr uint32_t kFixRangeHi = 0x40400000u;               // high word of 32.0

__device__ __forceinline__ long long pair_fix_raw(double x) {
  return __double_as_longlong(fma(x, 0x1p46, 0x1.8p52));
}

__device__ __forceinline__ void pair_fix_range(double x, uint32_t& hi_max) {
  hi_max = max(hi_max, (uint32_t)(__double_as_longlong(x) >> 32) & 0x7FFFFFFFu);
}

__device__ __forceinline__ double pair_fix_value(long long v) { return (double)v * 0x1p-46; }

// The same on the grid 2^-G (|x| < 2^(51-G)): pass A's forces and potential
// shares on 2^-40 (|term| < 2048), the Laplacian shares on 2^-30.
template <int G>
__device__ __forceinline__ long long fix_raw_g(double x) {
  return __double_as_longlong(fma(x, __builtin_ldexp(1.0, G), 0x1.8p52));
}
template <int G>
__device__ __forceinline__ double fix_value_g(long long v) {
  return (double)v * __builtin_ldexp(1.0, -G);
}
template <int G>
constexpr uint32_t fix_range_hi() {  // high word of 2^(51-G)
  return (uint32_t)(1023 + 51 - G) << 20;
}

// The tile of particle j relative to the tile starting at tb, or >= 128.
__device__ __forceinline__ uint32_t in_tile(uint32_t j, int64_t tb) {
  return j - (uint32_t)tb;
}

// Block status flag made uniform: one read, shared through LDS.
__device__ __forceinline__ bool block_status_set(const uint32_t* status, uint32_t* flag) {
  if (threadIdx.x == 0) *flag = *status;
  __syncthreads();
  return *flag != 0u;
}

// Conservative pair terms of one pair at squared distance r2 (r < rc), as
// seen by particle i: f * d_ij with f = -v'(r)/r, the potential v(r) and the
// Laplacian term v'' + 2 v'/r (eq. Tcon).  A coincident pair adds v(0) and
// no force.
template <int PREC>
__device__ __forceinline__ void pair_conservative(const Phys& P, double dx, double dy, double dz,
                                                  double r2, double& gx, double& gy, double& gz,
                                                  double& v, double& lap) {
  if constexpr (PREC == PREC_F64) {
    const double ir = inv_sqrt_f64(r2);  // 0 at r = 0
    const double rr = r2 * ir;
    double f;
    if (P.potential == 0) {
      const double w = 1.0 - rr * P.inv_rc;
      v = P.half_a_rc * w * w;
      f = P.a * w * ir;  // -v'(r)/r
      lap = ir > 0.0 ? P.a * P.inv_rc - 2.0 * P.a * w * ir : 0.0;
    } else {
      const double ir2 = ir * ir;
      const double s2 = P.r_lj2 * ir2;
      const double s6 = s2 * s2 * s2, s12 = s6 * s6;
      v = P.lj4e * (s12 - s6) - P.lj_vc - P.lj_dvc * (rr - P.rc);
      const double dv = -6.0 * P.lj4e * (2.0 * s12 - s6) * ir - P.lj_dvc;
      f = -dv * ir;
      lap = P.lj4e * (156.0 * s12 - 42.0 * s6) * ir2 + 2.0 * dv * ir;
    }
    gx = f * dx;
    gy = f * dy;
    gz = f * dz;
  } else {
    const float inv_rc_f = (float)P.inv_rc, a_f = (float)P.a;
    const float rr = __builtin_sqrtf((float)r2);
    const float ir = rr > 0.0f ? 1.0f / rr : 0.0f;
    float f;
    if (P.potential == 0) {
      const float w = 1.0f - rr * inv_rc_f;
      v = (double)((float)P.half_a_rc * w * w);
      f = a_f * w * ir;
      lap = (double)(rr > 0.0f ? a_f * inv_rc_f - 2.0f * a_f * w * ir : 0.0f);
    } else {
      const float ir2 = ir * ir;
      const float s2 = (float)P.r_lj2 * ir2;
      const float s6 = s2 * s2 * s2, s12 = s6 * s6;
      const float e4 = (float)P.lj4e;
      v = (double)(e4 * (s12 - s6) - (float)P.lj_vc - (float)P.lj_dvc * (rr - (float)P.rc));
      const float dv = -6.0f * e4 * (2.0f * s12 - s6) * ir - (float)P.lj_dvc;
      f = -dv * ir;
      lap = (double)(e4 * (156.0f * s12 - 42.0f * s6) * ir2 + 2.0f * dv * ir);
    }
    gx = (double)(f * (float)dx);
    gy = (double)(f * (float)dy);
    gz = (double)(f * (float)dz);
  }
}

// Pass A in the tile form: the tile's 128 particles, four lanes each, walk
// their skin lists (which hold the pairs tile_listed assigns them); every
// pair with r < rc goes to the work list of the step and its conservative
// terms are added once, in fixed point, to both particles (the partner's
// share through LDS when it lies in the tile; a pair joining two tiles is in
// both lists and adds to its own particle only).  Forces and potential shares
// (U_i = 1/2 sum_j v(r_ij)) on the grid 2^-g chosen from a (2^-46 for a < 16,
// 2^-45 for a = 25): the form is used with the soft potential, whose pair
// force and potential are bounded by a;
// the Laplacian shares, which grow as 1/r, in two words: the term on the grid
// 2^-20 and its remainder on 2^-50.  Mode 1 also applies p += dt/2 F (end of
// velocity-Verlet).
constexpr int kTileListLds = 16;  // work-list entries per particle staged in LDS
constexpr int kTileSkinLds = 28;  // skin-list entries per particle staged in LDS (a block loads every row)

// In a batch a wave walks its particles one replica at a time, with that
// replica's geometry uniform (in scalar registers).  Replicas of at least a
// wave's 16 particles (SMALL false) let a wave meet at most two, walked in
// straight-line code; with smaller ones (SMALL) a loop takes as many as the
// wave meets, at the cost of registers.
template <bool BATCH, int PREC, bool SMALL = false>
__global__ __launch_bounds__(kSub * kUniqTile) __attribute__((amdgpu_waves_per_eu(BATCH && SMALL ? 4 : 6, 8))) void k_pass_a_uniq(
    PState s, int64_t n, const Geo* __restrict__ geo, Phys P, int mode,
    double* __restrict__ Fx, double* __restrict__ Fy, double* __restrict__ Fz,
    double* __restrict__ Ui, double* __restrict__ Li, SkinList sl, NList nl, uint32_t* status) {
  constexpr int GH = 20, GR = 50;
  const double fsc = P.fix_scale_f;  // forces and potential shares: grid 1/fsc
  auto fix_f = [&](double x) { return __double_as_longlong(fma(x, fsc, 0x1.8p52)); };
  __shared__ unsigned long long acc[6][kUniqTile];  // Fx Fy Fz U Lhi Llo, two's complement
  __shared__ uint32_t lst[kTileListLds * kUniqTile];
  __shared__ uint32_t skin[kTileSkinLds * kUniqTile];  // the tile's skin lists, entry-major
  __shared__ uint32_t st_flag;
  for (int c = threadIdx.x; c < 6 * kUniqTile; c += blockDim.x) acc[c / kUniqTile][c % kUniqTile] = 0;
  if (block_status_set(status, &st_flag)) return;  // uniform in the block
  const int64_t tb = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * kUniqTile;
  {
    // the first kTileSkinLds entries of every skin list of the tile, loaded
    // row by row (128 consecutive words per row), all loads in flight at once
    constexpr int kPer = kTileSkinLds * kUniqTile / (kSub * kUniqTile);
    uint32_t v[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int c = r * (kSub * kUniqTile) + threadIdx.x;
      const int k = c / kUniqTile, t = c % kUniqTile;
      const int64_t row = tb + t < n ? tb + t : n - 1;
      v[r] = sl.idx[(int64_t)k * sl.stride + row];
    }
#pragma unroll
    for (int r = 0; r < kPer; ++r) skin[r * (kSub * kUniqTile) + threadIdx.x] = v[r];
    __syncthreads();
  }
  const int pl = threadIdx.x / kSub, sub = threadIdx.x % kSub;
  const int shift = (threadIdx.x % kWave) & ~(kSub - 1);
  const int64_t i = tb + pl;
  const bool live = i < n;
  const Rec* __restrict__ R = s.r;
  double xi = 0.0, yi = 0.0, zi = 0.0;
  uint32_t ns = 0, rep = 0u;
  if (live) {
    xi = R[i].qx;
    yi = R[i].qy;
    zi = R[i].qz;
    ns = sl.count[i];
    if constexpr (BATCH) rep = R[i].rep;
  }
  const uint32_t cap = (uint32_t)P.cap;
  long long XF0 = 0, XF1 = 0, XF2 = 0, XU = 0, XLh = 0, XLl = 0;  // raw fixed-point words
  long long terms = 0;
  uint32_t hi_l = 0u;
  uint32_t nn = 0;
  // The walk of the lanes in `mine` over their lists, with the geometry g of
  // their replica uniform in the wave (every pair term is a fixed-point sum,
  // so splitting a wave between replicas leaves the results' bits alone).
  auto walk = [&](const Geo& g, bool mine) {
    const bool mi = !__all(!mine || away_from_faces(g, P, xi, yi, zi));  // uniform in the wave
    if (!mine) return;
    // one trip of the group over entries base + sub (uniform in the group)
    auto trip = [&](uint32_t k, uint32_t j, double qjx, double qjy, double qjz) {
      bool take = false;
      double dx = 0.0, dy = 0.0, dz = 0.0, r2 = 0.0;
      if (k < ns) {
        separation_mi(g, mi, xi, yi, zi, qjx, qjy, qjz, dx, dy, dz);
        r2 = dist2(dx, dy, dz);
        take = r2 < P.rc2;
      }
      const uint32_t bits = (uint32_t)(__ballot(take) >> shift) & kSubMask;
      if (take) {
        const uint32_t pos = nn + __popc(bits & ((1u << sub) - 1u));
        if (pos < (uint32_t)kTileListLds) lst[pos * kUniqTile + pl] = j;
        else if (pos < cap) nl.idx[(int64_t)pos * nl.stride + i] = j;
        double gx, gy, gz, v, lap;
        pair_conservative<PREC>(P, dx, dy, dz, r2, gx, gy, gz, v, lap);
        const long long f0 = fix_f(gx), f1 = fix_f(gy), f2 = fix_f(gz);
        const long long fu = fix_f(0.5 * v);
        // Laplacian term: 2^-20 grid, then the (exact) remainder on 2^-50
        const long long fh = fix_raw_g<GH>(lap);
        const double rem = lap - (double)(fh - kFixMagicBits) * 0x1p-20;
        const long long fr = fix_raw_g<GR>(rem);
        // forces and potential shares are within the grid's range by its
        // choice (|f d| <= a, v/2 <= a rc/4); the Laplacian share grows as 1/r
        pair_fix_range(lap, hi_l);
        XF0 += f0;
        XF1 += f1;
        XF2 += f2;
        XU += fu;
        XLh += fh;
        XLl += fr;
        ++terms;
        const uint32_t rel = in_tile(j, tb);
        if (rel < (uint32_t)kUniqTile) {  // the partner's share of a pair inside the tile
          atomicAdd(&acc[0][rel], (unsigned long long)(kFixMagicBits - f0));
          atomicAdd(&acc[1][rel], (unsigned long long)(kFixMagicBits - f1));
          atomicAdd(&acc[2][rel], (unsigned long long)(kFixMagicBits - f2));
          atomicAdd(&acc[3][rel], (unsigned long long)(fu - kFixMagicBits));
          atomicAdd(&acc[4][rel], (unsigned long long)(fh - kFixMagicBits));
          atomicAdd(&acc[5][rel], (unsigned long long)(fr - kFixMagicBits));
        }
      }
      nn += __popc(bits);
    };
    // entries staged in LDS: the next trip's position is requested before
    // this trip's pair terms
    const uint32_t ns0 = ns < (uint32_t)kTileSkinLds ? ns : (uint32_t)kTileSkinLds;
    uint32_t jn = (uint32_t)sub < ns0 ? skin[sub * kUniqTile + pl] : 0u;
    double qnx = 0.0, qny = 0.0, qnz = 0.0;
    if ((uint32_t)sub < ns0) {
      qnx = R[jn].qx;
      qny = R[jn].qy;
      qnz = R[jn].qz;
    }
    uint32_t base = 0;
    for (; base < ns0; base += kSub) {
      const uint32_t k = base + sub;
      const uint32_t j = jn;
      const double qjx = qnx, qjy = qny, qjz = qnz;
      if (k + kSub < ns0) {
        jn = skin[(k + kSub) * kUniqTile + pl];
        qnx = R[jn].qx;
        qny = R[jn].qy;
        qnz = R[jn].qz;
      }
      trip(k, j, qjx, qjy, qjz);
    }
    // longer lists: the rest from memory
    for (; base < ns; base += kSub) {
      const uint32_t k = base + sub;
      uint32_t j = 0u;
      double qjx = 0.0, qjy = 0.0, qjz = 0.0;
      if (k < ns) {
        j = sl.idx[(int64_t)k * sl.stride + i];
        qjx = R[j].qx;
        qjy = R[j].qy;
        qjz = R[j].qz;
      }
      trip(k, j, qjx, qjy, qjz);
    }
  };
  if constexpr (BATCH && SMALL) {
    bool todo = live;
    while (__any(todo)) {
      const uint32_t r = (uint32_t)__builtin_amdgcn_readlane((int)rep, __builtin_ctzll(__ballot(todo)));
      const bool mine = todo && rep == r;
      walk(geo[r], mine);
      todo = todo && !mine;
    }
  } else if constexpr (BATCH) {
    // the wave's first replica, then the next one if the wave reaches it
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)rep);
    walk(geo[r0], live && rep == r0);
    const bool rest = live && rep != r0;
    if (__any(rest)) {
      const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)rep, __builtin_ctzll(__ballot(rest)));
      walk(geo[r1], rest);
    }
  } else {
    walk(geo[0], live);
  }
  const long long m = terms * kFixMagicBits;
  XF0 -= m;
  XF1 -= m;
  XF2 -= m;
  XU -= m;
  XLh -= m;
  XLl -= m;
#pragma unroll
  for (int off = 1; off < kSub; off <<= 1) {
    XF0 += __shfl_xor(XF0, off, kWave);
    XF1 += __shfl_xor(XF1, off, kWave);
    XF2 += __shfl_xor(XF2, off, kWave);
    XU += __shfl_xor(XU, off, kWave);
    XLh += __shfl_xor(XLh, off, kWave);
    XLl += __shfl_xor(XLl, off, kWave);
  }
  if (hi_l >= fix_range_hi<GH>()) atomicOr(status, ST_RANGE);
  __syncthreads();
  if (!live) return;
  if (nn > cap) {
    if (sub == 0) atomicOr(status, ST_OVERFLOW);
    nn = cap;
  }
  const uint32_t staged = nn < (uint32_t)kTileListLds ? nn : (uint32_t)kTileListLds;
  for (uint32_t k = sub; k < staged; k += kSub)
    nl.idx[(int64_t)k * nl.stride + i] = lst[k * kUniqTile + pl];
  if (sub == 0) {
    const double fx = (double)(long long)((unsigned long long)XF0 + acc[0][pl]) * P.fix_inv_f;
    const double fy = (double)(long long)((unsigned long long)XF1 + acc[1][pl]) * P.fix_inv_f;
    const double fz = (double)(long long)((unsigned long long)XF2 + acc[2][pl]) * P.fix_inv_f;
    nl.count[i] = nn;
    Fx[i] = fx;
    Fy[i] = fy;
    Fz[i] = fz;
    Ui[i] = (double)(long long)((unsigned long long)XU + acc[3][pl]) * P.fix_inv_f;
    Li[i] = fix_value_g<GH>((long long)((unsigned long long)XLh + acc[4][pl])) +
            fix_value_g<GR>((long long)((unsigned long long)XLl + acc[5][pl]));
    if (mode) {
      Rec* W = s.r;
      W[i].px = W[i].px + P.half_dt * fx;
      W[i].py = W[i].py + P.half_dt * fy;
      W[i].pz = W[i].pz + P.half_dt * fz;
    }
  }
}

// A wave of the tile sweeps serves 32 particles, two lanes each.  The first
// kTileRegular entries of every list go through the lane-pair loop; the
// entries beyond them, few and unevenly spread over the particles, are dealt
// evenly over all 64 lanes of the wave, so the wave does not wait for its
// longest list.
constexpr int kTileRegular = 8;

// The particle (0..31 within the wave) of overflow item x: the last p with
// first[p] <= x, first[] ascending in LDS.
__device__ __forceinline__ int overflow_owner(const uint32_t* first, uint32_t x) {
  int lo = 0, hi = 31;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Occupancy: the batched FP64 vector-model instance, which holds its
// replica's geometry per lane, fits 6 waves per SIMD only when asked (79
// VGPRs, no spills); asked the same, the FP32 and projected-model instances
// would spill, and keep the compiler's choice.
template <bool BATCH, int PREC, int MODEL>
__global__ __launch_bounds__(2 * kUniqTile)
__attribute__((amdgpu_waves_per_eu(BATCH && PREC == PREC_F64 && MODEL == 0 ? 6 : 1, 8)))
void k_pass_b_uniq(
    PState s, NList nl, int64_t n, const Geo* __restrict__ geo, Phys P,
    const uint64_t* __restrict__ d_step, Vec4* __restrict__ dpi, H3* __restrict__ hv, int store,
    uint32_t* status) {
  // two's-complement sums in unsigned words (the atomic add is modular)
  __shared__ unsigned long long acc[3][kUniqTile];
  __shared__ uint32_t first_s[2 * kUniqTile / kWave][32];
  __shared__ uint32_t st_flag;
  for (int c = threadIdx.x; c < 3 * kUniqTile; c += blockDim.x) acc[c / kUniqTile][c % kUniqTile] = 0;
  if (block_status_set(status, &st_flag)) return;  // uniform in the block
  const int64_t tb = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * kUniqTile;
  const int pl = threadIdx.x >> 1, sub = threadIdx.x & 1;
  const int w = threadIdx.x / kWave;
  uint32_t* first = first_s[w];
  const int64_t i = tb + pl;
  const bool live = i < n;
  const uint64_t step = *d_step;
  const Rec* __restrict__ R = s.r;
  const int64_t st = nl.stride;
  long long X0 = 0, X1 = 0, X2 = 0;  // raw sums of fixed-point bit patterns
  long long terms = 0;
  uint32_t hi_max = 0u;
  Rec a{};
  uint32_t nn = 0;
  bool away = true;
  if (live) {
    a = R[i];
    nn = nl.count[i];
    const GeoRef<BATCH> g = geo[BATCH ? a.rep : 0u];
    away = away_from_faces(g, P, a.qx, a.qy, a.qz);
  }
  const bool mi = !__all(away);  // uniform in the wave
  // the pair term of entry k (partner j) of particle ii (record ra): stored,
  // its share added to the partner inside the tile; returns the raw
  // fixed-point words
  auto term = [&](const Rec& ra, int64_t ii, uint32_t k, uint32_t j, long long& f0,
                  long long& f1, long long& f2) {
    const int64_t e = (int64_t)k * st + ii;
    const Rec b = R[j];
    const GeoRef<BATCH> g = geo[BATCH ? ra.rep : 0u];
    double vx, vy, vz;
    PairOut o;
    pair_from_records<PREC, MODEL>(P, g, mi, ra, b, step, vx, vy, vz, o);
    if (store) store_dp<PREC>(nl, e, o.dp[0], o.dp[1], o.dp[2]);
    f0 = pair_fix_raw(o.dp[0]);
    f1 = pair_fix_raw(o.dp[1]);
    f2 = pair_fix_raw(o.dp[2]);
    pair_fix_range(o.dp[0], hi_max);
    pair_fix_range(o.dp[1], hi_max);
    pair_fix_range(o.dp[2], hi_max);
    const uint32_t rel = in_tile(j, tb);
    if (rel < (uint32_t)kUniqTile) {  // the partner's share of a pair inside the tile
      atomicAdd(&acc[0][rel], (unsigned long long)(kFixMagicBits - f0));
      atomicAdd(&acc[1][rel], (unsigned long long)(kFixMagicBits - f1));
      atomicAdd(&acc[2][rel], (unsigned long long)(kFixMagicBits - f2));
    }
  };
  const uint32_t nreg = nn < (uint32_t)kTileRegular ? nn : (uint32_t)kTileRegular;
  // this lane's regular entries sub, sub + 2, ...: every index load in flight
  // at once (addresses clamped to the list, so no load needs a branch)
  uint32_t jr[kTileRegular / 2];
#pragma unroll
  for (int q = 0; q < kTileRegular / 2; ++q) {
    const uint32_t k = (uint32_t)(sub + 2 * q);
    const uint32_t kc = k < nreg ? k : (nreg ? nreg - 1u : 0u);
    jr[q] = nreg ? nl.idx[(int64_t)kc * st + i] : 0u;
  }
  for (int q = 0; q < kTileRegular / 2; ++q) {
    const uint32_t k = (uint32_t)(sub + 2 * q);
    if (k >= nreg) break;
    long long f0, f1, f2;
    term(a, i, k, jr[q], f0, f1, f2);
    X0 += f0;
    X1 += f1;
    X2 += f2;
    ++terms;
  }
  // the entries beyond kTileRegular, dealt over the wave
  uint32_t total;
  const uint32_t extra = (sub == 0 && nn > (uint32_t)kTileRegular) ? nn - kTileRegular : 0u;
  const uint32_t pre = wave_prefix(extra, total);
  if (total) {  // uniform in the wave
    if (sub == 0) first[pl % 32] = pre;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    for (uint32_t x = threadIdx.x % kWave; x < total; x += kWave) {
      const int p = overflow_owner(first, x);
      const int slot = 32 * w + p;
      const int64_t ii = tb + slot;
      const uint32_t k = (uint32_t)kTileRegular + (x - first[p]);
      const Rec ra = R[ii];
      long long f0, f1, f2;
      term(ra, ii, k, nl.idx[(int64_t)k * st + ii], f0, f1, f2);
      atomicAdd(&acc[0][slot], (unsigned long long)(f0 - kFixMagicBits));
      atomicAdd(&acc[1][slot], (unsigned long long)(f1 - kFixMagicBits));
      atomicAdd(&acc[2][slot], (unsigned long long)(f2 - kFixMagicBits));
    }
  }
  X0 -= terms * kFixMagicBits;
  X1 -= terms * kFixMagicBits;
  X2 -= terms * kFixMagicBits;
  X0 += __shfl_xor(X0, 1, kWave);
  X1 += __shfl_xor(X1, 1, kWave);
  X2 += __shfl_xor(X2, 1, kWave);
  if (hi_max >= kFixRangeHi) atomicOr(status, ST_RANGE);
  __syncthreads();
  if (!live || sub) return;
  const double ax = pair_fix_value((long long)((unsigned long long)X0 + acc[0][pl]));
  const double ay = pair_fix_value((long long)((unsigned long long)X1 + acc[1][pl]));
  const double az = pair_fix_value((long long)((unsigned long long)X2 + acc[2][pl]));
  dpi[i] = Vec4{ax, ay, az, 0.0};
  hv[i] = H3{fma(ax, P.inv_2m, a.px * P.inv_mass), fma(ay, P.inv_2m, a.py * P.inv_mass),
             fma(az, P.inv_2m, a.pz * P.inv_mass)};
}

// ---------------------------------------------------------------------------
// Inverse temperature of the updated internal energy.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double inv_temperature(const Phys& P, double eps, uint32_t* status) {
  if (P.eos == 0) return P.cv / eps;
  int it;
  const double th = theta_newton_dev(P, eps, theta_start_dev(P, eps), it);
  if (!(th > 0.0) || !isfinite(th)) atomicOr(status, ST_EOS);
  return 1.0 / th;
}

// ---------------------------------------------------------------------------
// Pass C (SER sweep 2): d eps_i = -1/2 sum_j dp_ij . (v_ij + (dp_i - dp_j)/(2m))
// in FP64 for both precisions, then p <- p + dp, eps <- eps + d eps and the
// next 1/T_i.  The new records go to `out`, never over the records this pass
// gathers from.
// ---------------------------------------------------------------------------
// THETA = 1: the surrogate network gives the next 1/T_i inside this pass
// (the learned-EOS modes): the block's particles put their inputs in LDS,
// one wave evaluates the network for all of them on the matrix cores, and
// each particle finishes as the stand-alone theta kernel does (Newton outside
// the training range).  The block therefore meets at barriers and takes no
// early exit before them.
template <bool BATCH, int PREC, int REGEN, int MODEL, int THETA>
__global__ __launch_bounds__(kPairBlockMax) void k_pass_c(
    PState s, NList nl, int64_t n, const Geo* __restrict__ geo, Phys P,
    const uint64_t* __restrict__ d_step, const Vec4* __restrict__ dpi,
    const H3* __restrict__ hv, int eos_inline, MlpDev m, int mlp_mode, Rec* __restrict__ out,
    uint32_t* status) {
  __shared__ float net_x[kPairBlockMax / kSubSer];
  __shared__ float net_y[kPairBlockMax / kSubSer];
  __shared__ uint32_t st_flag;
  const Lanes L = lanes<kSubSer>();
  const bool live = L.i < n;  // uniform in the group
  if constexpr (THETA) {
    if (threadIdx.x == 0) st_flag = *status;
    __syncthreads();
    if (st_flag) return;  // uniform in the block
  } else {
    if (!live) return;
    if (status_set(status)) return;
  }
  const int64_t i = live ? L.i : 0;
  double de = 0.0;
  Rec a{};
  Vec4 di{};
  if (live) {
    const uint64_t step = *d_step;
    const Rec* __restrict__ R = s.r;
    a = R[i];
    const GeoRef<BATCH> g = geo[BATCH ? a.rep : 0u];
    const bool mi = REGEN ? !__all(away_from_faces(g, P, a.qx, a.qy, a.qz)) : true;
    di = dpi[i];
    const H3 hi = hv[i];
    const uint32_t nn = nl.count[i];
    const int64_t st = nl.stride;
    uint32_t jn = (uint32_t)L.sub < nn ? nl.idx[(int64_t)L.sub * st + i] : 0u;
    double hx = 0.0, hy = 0.0, hz = 0.0;
    if ((uint32_t)L.sub < nn) {
      hx = hv[jn].x;
      hy = hv[jn].y;
      hz = hv[jn].z;
    }
    for (uint32_t k = L.sub; k < nn; k += kSubSer) {
      const int64_t e = (int64_t)k * st + i;
      const uint32_t j = jn;
      const double ux = hi.x - hx, uy = hi.y - hy, uz = hi.z - hz;
      if (k + kSubSer < nn) {
        jn = nl.idx[e + kSubSer * st];
        hx = hv[jn].x;
        hy = hv[jn].y;
        hz = hv[jn].z;
      }
      double ex, ey, ez;
      if constexpr (REGEN) {
        const Rec b = R[j];
        double vx, vy, vz;
        PairOut o;
        pair_from_records<PREC, MODEL>(P, g, mi, a, b, step, vx, vy, vz, o);
        ex = o.dp[0];
        ey = o.dp[1];
        ez = o.dp[2];
      } else {
        load_dp<PREC>(nl, e, ex, ey, ez);
      }
      de += -0.5 * (ex * ux + ey * uy + ez * uz);
    }
    de = group_sum<kSubSer>(de);
  }
  const double e = live ? s.eps[i] + de : 1.0;
  // The record (with the old 1/T_i) is written before the network, so that
  // only e and i stay live across it; the new 1/T_i follows.
  const bool own = live && L.sub == 0;
  bool need_t = false;
  if (own) {
    Rec o = a;
    o.px = a.px + di.x;
    o.py = a.py + di.y;
    o.pz = a.pz + di.z;
    s.eps[i] = e;
    if (!(e > 0.0)) {
      atomicOr(status, ST_NEG_EINT);
    } else if constexpr (THETA) {
      need_t = true;
    } else if (eos_inline) {
      o.invT = inv_temperature(P, e, status);
    }
    out[i] = o;
  }
  if constexpr (THETA) {
    float y = 0.0f;
    if (mlp_mode != 0) {  // uniform
      if (L.sub == 0) net_x[L.pib] = mlp_input(m, e);
      __syncthreads();
      // wave w takes particles 32 w .. 32 w + 31 of the block
      const int w = threadIdx.x / kWave, col = threadIdx.x % 32;
      if (32 * w < L.ppb) {  // uniform in the wave
        const int p = 32 * w + col;
        const float yw = mlp_wave32(m.wf, m.wb, p < L.ppb ? net_x[p] : 0.0f);
        if (threadIdx.x % kWave < 32) net_y[p] = yw;
      }
      __syncthreads();
      y = net_y[L.pib];
    }
    if (need_t) {
      int it;
      const double th = theta_from_net(P, m, mlp_mode, e, y, it);
      if (!(th > 0.0) || !isfinite(th)) atomicOr(status, ST_EOS);
      out[i].invT = 1.0 / th;
    }
  }
}

// Observables of a step (the energy of Sec. 2.1, the temperatures of
// Sec. 2.2) are sums over particles of
// U, K, sum eps, Px, Py, Pz, sum 1/T, |grad U|^2, Laplacian U, out-of-range count
constexpr int kStatVals = 10;
constexpr int kStatBad = 9;
constexpr int kRecLen = 12;  // record: U K sum-eps E Px Py Pz Tkin Tint n |gradU|^2 lapU

// The per-particle terms of those sums, defined once so that both producers
// of the partial sums give the same bits.
__device__ __forceinline__ double sq3(double x, double y, double z) {
  return x * x + y * y + z * z;
}
__device__ __forceinline__ double kinetic(double px, double py, double pz, double mass) {
  return sq3(px, py, pz) / (2.0 * mass);
}
// A value's fixed-point form; a value outside the range adds one to the
// out-of-range count instead (the record is then NaN).
__device__ __forceinline__ Fix stat_fix(double x, int& bad) {
  if (fabs(x) < 0x1p30) return fix_of(x);
  ++bad;
  return fix_zero();
}

// The end of a step fused into the tile sweep 2: each tile's partial sums of
// the finished step's observables, and the next step's kick and drift on the
// records it writes, with the maxima of that step's list-build decision.
// Kicking requires the sums (the separate observables pass reads the
// records, which would then be kicked).  In a batch every replica holds at
// least a tile's particles, so a tile spans at most two replicas.
struct StepTail {
  const double* Fx;  // F of the step (pass A)
  const double* Fy;
  const double* Fz;
  const double* Ui;  // per-particle shares of U and of its Laplacian
  const double* Li;
  const QIdF* ref;   // positions at the last list build (FP32)
  BuildCtl* next;    // the next step's maxima; the step's end moves them into the build control
  Fix* partials;     // kStatVals per slot, cleared by their reader
  int slots;         // slots per replica: tile t adds into slot t % slots of its replica(s)
  int stats;         // add the partial sums
  int kick;          // kick and drift the written records
};

// Slots of the partial sums: tiles in flight together (consecutive ones) add
// into different slots, and the final pass reads two per lane; a batch's
// replicas take a few each.
constexpr int kTailSlots = 128;
constexpr int kTailSlotsPerReplica = 4;

// dst += v exactly, in any order of the adds to dst: the low words add
// modulo 2^64, and the add that wraps them (known from the old value the
// atomic returns) carries one into the high word.
__device__ __forceinline__ void fix_atomic_add(Fix* dst, Fix v) {
  unsigned long long* lo = reinterpret_cast<unsigned long long*>(&dst->lo);
  unsigned long long* hi = reinterpret_cast<unsigned long long*>(&dst->hi);
  const unsigned long long old = atomicAdd(lo, (unsigned long long)v.lo);
  const unsigned long long carry = (old + (unsigned long long)v.lo < old) ? 1ull : 0ull;
  const unsigned long long h = (unsigned long long)v.hi + carry;
  if (h) atomicAdd(hi, h);
}

constexpr int kUniqWaves = 2 * kUniqTile / kWave;  // waves of a tile sweep's block

// One sum over the wave's even lanes and another over its odd lanes (the
// butterfly rounds never pair an even lane with an odd one); lanes 0 and 1
// store them as values ke and ko of wave w.
__device__ __forceinline__ void wave_pair_sums(Fix f, Fix (*out)[kUniqWaves], int ke, int ko,
                                               int w) {
#pragma unroll
  for (int off = kWave / 2; off > 1; off >>= 1) {
    Fix b;
    b.lo = (uint64_t)__shfl_xor((long long)f.lo, off, kWave);
    b.hi = (int64_t)__shfl_xor((long long)f.hi, off, kWave);
    f = fix_add(f, b);
  }
  const int lane = threadIdx.x % kWave;
  if (lane == 0) out[ke][w] = f;
  if (lane == 1) out[ko][w] = f;
}

// Pass C over the tile's unique pairs: the reinjection term
//   e_ij = -1/2 dp_ij . (h_i - h_j),   h = (p + dp/2)/m
// is symmetric in (i, j), so a pair inside the tile adds the same e_ij to both
// internal energies (eq. SER_eint_discretization); then p <- p + dp,
// eps <- eps + d eps and the next 1/T_i as in k_pass_c (THETA = 1: the
// surrogate network inside the pass); with a StepTail also the observables'
// partial sums and the next step's kick.  Occupancy, with stored
// increments: 6 waves per SIMD fit with the network (its registers are dead
// by the tail); the inline-EOS instances need 5 to keep the tail out of
// scratch.  The instances that regenerate the noise hold the pair term's
// registers as well and keep the compiler's choice (asked for 5 or 6 they
// spill).
template <bool BATCH, int PREC, int REGEN, int MODEL, int THETA>
__global__ __launch_bounds__(2 * kUniqTile)
__attribute__((amdgpu_waves_per_eu(REGEN ? 1 : (THETA ? 6 : 5), 8))) void k_pass_c_uniq(
    PState s, NList nl, int64_t n, const Geo* __restrict__ geo, Phys P,
    const uint64_t* __restrict__ d_step, const Vec4* __restrict__ dpi,
    const H3* __restrict__ hv, int eos_inline, MlpDev m, int mlp_mode, Rec* __restrict__ out,
    StepTail tail, uint32_t* status) {
  __shared__ unsigned long long acc[kUniqTile];  // two's-complement sums (modular adds)
  __shared__ float net_x[kUniqTile];
  __shared__ float net_y[kUniqTile];
  __shared__ uint32_t first_s[kUniqWaves][32];
  __shared__ double hs[3][kUniqTile];  // the tile's h: partners inside the tile read it here
  __shared__ Fix stat_s[BATCH ? 2 : 1][kStatVals][kUniqWaves];
  __shared__ uint32_t st_flag;
  for (int c = threadIdx.x; c < kUniqTile; c += blockDim.x) acc[c] = 0;
  const int64_t tb = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * kUniqTile;
  if (threadIdx.x < kUniqTile && tb + threadIdx.x < n) {
    const H3 h = hv[tb + threadIdx.x];
    hs[0][threadIdx.x] = h.x;
    hs[1][threadIdx.x] = h.y;
    hs[2][threadIdx.x] = h.z;
  }
  if (block_status_set(status, &st_flag)) return;  // uniform in the block (and hs visible)
  const int pl = threadIdx.x >> 1, sub = threadIdx.x & 1;
  const int w = threadIdx.x / kWave;
  uint32_t* first = first_s[w];
  const int64_t i = tb + pl;
  const bool live = i < n;
  const uint64_t step = *d_step;
  const Rec* __restrict__ R = s.r;
  const int64_t st = nl.stride;
  long long X = 0;  // raw sum of fixed-point bit patterns
  long long terms = 0;
  uint32_t hi_max = 0u;
  Rec a{};
  Vec4 di{};
  uint32_t nn = 0;
  bool away = true;
  if (live) {
    a = R[i];
    di = dpi[i];
    nn = nl.count[i];
    if constexpr (REGEN) {
      const GeoRef<BATCH> g = geo[BATCH ? a.rep : 0u];
      away = away_from_faces(g, P, a.qx, a.qy, a.qz);
    }
  }
  const bool mi = REGEN ? !__all(away) : true;  // uniform in the wave
  // h_j of a partner: from LDS inside the tile, else from memory
  auto gather_h = [&](uint32_t j, double& x, double& y, double& z) {
    const uint32_t rel = in_tile(j, tb);
    if (rel < (uint32_t)kUniqTile) {
      x = hs[0][rel];
      y = hs[1][rel];
      z = hs[2][rel];
    } else {
      const H3 h = hv[j];
      x = h.x;
      y = h.y;
      z = h.z;
    }
  };
  // e_ij of entry k of particle ii (record ra, h_i = hi), given the
  // partner's index j and h_j; its share added to the partner inside the tile
  // (dx, dy, dz: the stored increment when the caller has loaded it, with
  // `have`)
  auto term = [&](const Rec& ra, const H3& hi, int64_t ii, uint32_t k, uint32_t j, double hx,
                  double hy, double hz, bool have = false, double dx = 0.0, double dy = 0.0,
                  double dz = 0.0) -> long long {
    const int64_t e = (int64_t)k * st + ii;
    const double ux = hi.x - hx, uy = hi.y - hy, uz = hi.z - hz;
    double ex = dx, ey = dy, ez = dz;
    if constexpr (REGEN) {
      const Rec b = R[j];
      const GeoRef<BATCH> g = geo[BATCH ? ra.rep : 0u];
      double vx, vy, vz;
      PairOut o;
      pair_from_records<PREC, MODEL>(P, g, mi, ra, b, step, vx, vy, vz, o);
      ex = o.dp[0];
      ey = o.dp[1];
      ez = o.dp[2];
    } else {
      if (!have) load_dp<PREC>(nl, e, ex, ey, ez);
    }
    const double eij = -0.5 * (ex * ux + ey * uy + ez * uz);
    const long long f = pair_fix_raw(eij);
    pair_fix_range(eij, hi_max);
    const uint32_t rel = in_tile(j, tb);
    if (rel < (uint32_t)kUniqTile) atomicAdd(&acc[rel], (unsigned long long)(f - kFixMagicBits));
    return f;
  };
  if (live) {
    const H3 hi = hv[i];
    const uint32_t nreg = nn < (uint32_t)kTileRegular ? nn : (uint32_t)kTileRegular;
    // this lane's regular entries: every index load in flight at once, then
    // each partner's h requested one entry ahead
    uint32_t jr[kTileRegular / 2];
#pragma unroll
    for (int q = 0; q < kTileRegular / 2; ++q) {
      const uint32_t k = (uint32_t)(sub + 2 * q);
      const uint32_t kc = k < nreg ? k : (nreg ? nreg - 1u : 0u);
      jr[q] = nreg ? nl.idx[(int64_t)kc * st + i] : 0u;
    }
    double hx = 0.0, hy = 0.0, hz = 0.0;
    double sx = 0.0, sy = 0.0, sz = 0.0;  // the stored increment, likewise one entry ahead
    if ((uint32_t)sub < nreg) {
      gather_h(jr[0], hx, hy, hz);
      if constexpr (!REGEN) load_dp<PREC>(nl, (int64_t)sub * st + i, sx, sy, sz);
    }
#pragma unroll
    for (int q = 0; q < kTileRegular / 2; ++q) {
      const uint32_t k = (uint32_t)(sub + 2 * q);
      if (k >= nreg) break;
      const double cx = hx, cy = hy, cz = hz;
      const double ex = sx, ey = sy, ez = sz;
      if (q + 1 < kTileRegular / 2 && k + 2 < nreg) {
        gather_h(jr[q + 1], hx, hy, hz);
        if constexpr (!REGEN) load_dp<PREC>(nl, (int64_t)(k + 2) * st + i, sx, sy, sz);
      }
      X += term(a, hi, i, k, jr[q], cx, cy, cz, !REGEN, ex, ey, ez);
      ++terms;
    }
  }
  // the entries beyond kTileRegular, dealt over the wave
  uint32_t total;
  const uint32_t extra = (sub == 0 && nn > (uint32_t)kTileRegular) ? nn - kTileRegular : 0u;
  const uint32_t pre = wave_prefix(extra, total);
  if (total) {  // uniform in the wave
    if (sub == 0) first[pl % 32] = pre;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    for (uint32_t x = threadIdx.x % kWave; x < total; x += kWave) {
      const int p = overflow_owner(first, x);
      const int slot = 32 * w + p;
      const int64_t ii = tb + slot;
      const uint32_t k = (uint32_t)kTileRegular + (x - first[p]);
      const uint32_t j = nl.idx[(int64_t)k * st + ii];
      const H3 hj = hv[j];
      const Rec ra = REGEN ? R[ii] : Rec{};
      const long long f = term(ra, hv[ii], ii, k, j, hj.x, hj.y, hj.z);
      atomicAdd(&acc[slot], (unsigned long long)(f - kFixMagicBits));
    }
  }
  X -= terms * kFixMagicBits;
  X += __shfl_xor(X, 1, kWave);
  if (hi_max >= kFixRangeHi) atomicOr(status, ST_RANGE);
  __syncthreads();
  const double de =
      live ? pair_fix_value((long long)((unsigned long long)X + acc[pl])) : 0.0;
  const double e = live ? s.eps[i] + de : 1.0;
  // The record (with the old 1/T_i) is written before the network, so that
  // only e and i stay live across it; the new 1/T_i follows.
  const bool own = live && sub == 0;
  bool need_t = false;
  // the particle's updated record, formed on both of its lanes; the first
  // lane writes it
  Rec o = a;
  o.px = a.px + di.x;
  o.py = a.py + di.y;
  o.pz = a.pz + di.z;
  if (own) {
    s.eps[i] = e;
    if (!(e > 0.0)) {
      atomicOr(status, ST_NEG_EINT);
    } else if constexpr (THETA) {
      need_t = true;
    } else if (eos_inline) {
      o.invT = inv_temperature(P, e, status);
    }
  }
  // The finished step's observables: the particle's values split over its
  // two lanes (first lane: U, sum eps, Py, |grad U|^2, 1/T; second: K, Px,
  // Pz, Laplacian U and the particle's out-of-range count), each pair summed
  // over the wave's first and second lanes apart.
  // A batch's tile: the replica of its first particle (set 0) and, when the
  // last one differs, the next replica (set 1).
  int bad = 0;
  double F[3] = {0.0, 0.0, 0.0};
  const bool ev = sub == 0;
  uint32_t rep0 = 0u, rep1 = 0u;
  if constexpr (BATCH) {
    if (tail.stats) {
      rep0 = R[tb].rep;
      rep1 = R[(tb + kUniqTile < n ? tb + kUniqTile : n) - 1].rep;
    }
  }
  const bool two = rep1 != rep0;
  const bool in0 = !BATCH || a.rep == rep0;
  auto sums = [&](Fix f, int ke, int ko) {
    wave_pair_sums(in0 ? f : fix_zero(), stat_s[0], ke, ko, w);
    if constexpr (BATCH) {
      if (two) wave_pair_sums(in0 ? fix_zero() : f, stat_s[1], ke, ko, w);
    }
  };
  if ((tail.stats || tail.kick) && live) {
    F[0] = tail.Fx[i];
    F[1] = tail.Fy[i];
    F[2] = tail.Fz[i];
  }
  if (tail.stats) {  // uniform
    auto put = [&](double xe, double xo, int ke, int ko) {
      sums(live ? stat_fix(ev ? xe : xo, bad) : fix_zero(), ke, ko);
    };
    put(live && ev ? tail.Ui[i] : 0.0, kinetic(o.px, o.py, o.pz, P.mass), 0, 1);
    put(e, o.px, 2, 3);
    put(o.py, o.pz, 4, 5);
    put(sq3(F[0], F[1], F[2]), live && !ev ? tail.Li[i] : 0.0, 7, 8);
  }
  if (tail.kick) {  // uniform: the next step's first half-kick and drift
    double d2 = 0.0, qa = 0.0;
    if (own) {
      const GeoRef<BATCH> g = geo[BATCH ? a.rep : 0u];
      kick_record(o, F, g, P, 1, tail.ref, i, d2, qa, status);
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) d2 = fmax(d2, __shfl_xor(d2, off, kWave));
    if (threadIdx.x % kWave == 0) raise_max_bits(&tail.next->dmax_bits, d2);
    if (__any(qa > 0.0)) {
#pragma unroll
      for (int off = kWave / 2; off > 0; off >>= 1) qa = fmax(qa, __shfl_xor(qa, off, kWave));
      if (threadIdx.x % kWave == 0) raise_max_bits(&tail.next->qmax_bits, qa);
    }
  }
  // The record (with the old 1/T_i when the network follows) is written
  // before the network, so that only e and i stay live across it; the new
  // 1/T_i follows.
  if (own) out[i] = o;
  double inv_t = o.invT;
  if constexpr (THETA) {
    float y = 0.0f;
    if (mlp_mode != 0) {  // uniform
      if (sub == 0) net_x[pl] = mlp_input(m, e);
      __syncthreads();
      // wave w takes particles 32 w .. 32 w + 31 of the tile
      const int col = threadIdx.x % 32;
      const float yw = mlp_wave32(m.wf, m.wb, net_x[32 * w + col]);
      if (threadIdx.x % kWave < 32) net_y[32 * w + col] = yw;
      __syncthreads();
      y = net_y[pl];
    }
    if (need_t) {
      int it;
      const double th = theta_from_net(P, m, mlp_mode, e, y, it);
      if (!(th > 0.0) || !isfinite(th)) atomicOr(status, ST_EOS);
      inv_t = 1.0 / th;
      out[i].invT = inv_t;
    }
  }
  if (tail.stats) {  // uniform: 1/T and the out-of-range count, then the block's sums
    const Fix ft = live && ev ? stat_fix(inv_t, bad) : fix_zero();
    const int nbad = bad + __shfl_xor(bad, 1, kWave);  // both lanes of the particle
    sums(ev ? ft : Fix{(uint64_t)(uint32_t)nbad, 0ll}, 6, kStatBad);
    __syncthreads();
    if (threadIdx.x < (two ? 2 : 1) * kStatVals) {
      const int set = threadIdx.x / kStatVals, k = threadIdx.x % kStatVals;
      Fix t = fix_zero();
#pragma unroll
      for (int q = 0; q < kUniqWaves; ++q) t = fix_add(t, stat_s[BATCH ? set : 0][k][q]);
      const int64_t slot =
          (int64_t)(set ? rep1 : rep0) * tail.slots + (tb / kUniqTile) % tail.slots;
      fix_atomic_add(&tail.partials[slot * kStatVals + k], t);
    }
  }
}

// SEM: apply dp and d eps (both from pass B), then the next 1/T_i.
__global__ void k_apply_sem(PState s, int64_t n, Phys P, const Vec4* __restrict__ dpi,
                            const double* __restrict__ deps, int eos_inline,
                            Rec* __restrict__ out, uint32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (status_set(status)) return;
  Rec o = s.r[i];
  const Vec4 d = dpi[i];
  o.px += d.x;
  o.py += d.y;
  o.pz += d.z;
  const double e = s.eps[i] + deps[i];
  s.eps[i] = e;
  if (!(e > 0.0)) {
    atomicOr(status, ST_NEG_EINT);
  } else if (eos_inline) {
    o.invT = inv_temperature(P, e, status);
  }
  out[i] = o;
}

// 1/T_i for every particle (initialisation and the separate-EOS path).
__global__ void k_inv_temperature(PState s, int64_t n, Phys P, uint32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double e = s.eps[i];
  if (!(e > 0.0)) {
    atomicOr(status, ST_NEG_EINT);
    return;
  }
  s.r[i].invT = inv_temperature(P, e, status);
}

// ---------------------------------------------------------------------------
// Observables: per-tile partial sums (k_stats_tiles, or the end of the tile
// sweep 2), then one block per replica, all in the fixed-point form above, so
// a record does not depend on the particles' memory order (list rebuild
// schedule, batching, resume).
// Record: U, K, sum eps, E, Px, Py, Pz, T_kin, T_int, step.
// ---------------------------------------------------------------------------
constexpr int kStatThreads = 512;

__global__ __launch_bounds__(kStatThreads) void k_stats_tiles(
    PState s, const double* __restrict__ Ui, const double* __restrict__ Li,
    const double* __restrict__ Fx, const double* __restrict__ Fy, const double* __restrict__ Fz,
    const int64_t* __restrict__ tile_begin, Phys P, Fix* __restrict__ partials) {
  const int64_t b = tile_begin[blockIdx.x], e = tile_begin[blockIdx.x + 1];
  Fix v[kStatVals];
#pragma unroll
  for (int k = 0; k < kStatVals; ++k) v[k] = fix_zero();
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
    const Rec& rc = s.r[i];
    const double px = rc.px, py = rc.py, pz = rc.pz;
    const double x[9] = {Ui[i], kinetic(px, py, pz, P.mass), s.eps[i], px, py, pz, rc.invT,
                         sq3(Fx[i], Fy[i], Fz[i]), Li[i]};
    int bad = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) v[k] = fix_add(v[k], stat_fix(x[k], bad));
    v[kStatBad] = fix_add(v[kStatBad], Fix{(uint64_t)(uint32_t)bad, 0ll});
  }
  __shared__ Fix smem[kStatVals * (kStatThreads / kWave)];
  block_sum_fix<kStatVals>(v, smem);
  if (threadIdx.x == 0)
    for (int k = 0; k < kStatVals; ++k) partials[blockIdx.x * kStatVals + k] = v[k];
}

// End of the step: count a list build, reset the build control for the next
// step, advance the step and history counters (nothing but the reset of the
// next step's maxima when the status is raised).  The
// counters' values were read before (no other block writes them).
struct StepNow {
  uint64_t step;
  int64_t hist;
  unsigned long long builds;
  bool rebuilt, failed;
};

__device__ __forceinline__ void step_end(const StepNow& c, uint64_t* d_step, int64_t* d_hist_count,
                                         BuildCtl* ctl, BuildCtl* next,
                                         unsigned long long* builds, int advance) {
  // the next step's maxima (nonzero when its kick ran at the end of this
  // step's sweep 2) become the build control; the slot is left cleared
  const unsigned long long nd = next->dmax_bits, nq = next->qmax_bits;
  next->dmax_bits = 0ull;
  next->qmax_bits = 0ull;
  if (c.failed) return;
  if (c.rebuilt) *builds = c.builds + 1ull;
  ctl->dmax_bits = nd;
  ctl->force = 0u;
  ctl->qmax_bits = nq;
  if (advance) {
    *d_step = c.step + 1;
    *d_hist_count = c.hist + 1;
  }
}

// Per replica: sum the tile partials, write the record (and the history
// row); with `clear`, leave the partials zero (slots that the tile sweep 2
// adds into).  With `finish`, the last block to complete also ends the step: a
// ticket taken after each block's reads of the step and history counters
// tells it that every other block is done with them.
constexpr int kStatFinalThreads = kStatVals * kWave;  // one wave per recorded sum

__global__ __launch_bounds__(kStatFinalThreads) void k_stats_final(
    Fix* __restrict__ partials, int clear, const int32_t* __restrict__ rep_tile0,
    const Geo* __restrict__ geo, uint64_t* d_step, int advance,
    double* __restrict__ rec, double* __restrict__ hist, int64_t hist_cap,
    int64_t* d_hist_count, int nrep, int finish, uint32_t* ticket, BuildCtl* ctl,
    BuildCtl* next, unsigned long long* builds, double half_skin2, const uint32_t* status) {
  const int r = blockIdx.x;
  const int t0 = rep_tile0[r], t1 = rep_tile0[r + 1];
  // the values the record and the end of the step need, requested before
  // the reduction so that their latency overlaps it
  StepNow now{*d_step, *d_hist_count, 0ull, false, false};
  if (finish) {
    now.builds = *builds;
    now.rebuilt = rebuild_now(ctl, half_skin2);
    now.failed = status_set(status);
  }
  const double N = (double)geo[r].n;
  // wave k adds value k over the replica's tiles
  const int k0 = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  // eight partials per lane in flight, then (with clear) their slots zeroed
  constexpr int kAhead = 8;
  Fix acc = fix_zero();
  for (int tb = t0 + lane; tb < t1; tb += kAhead * kWave) {
    Fix v[kAhead];
#pragma unroll
    for (int u = 0; u < kAhead; ++u) {
      const int t = tb + u * kWave;
      v[u] = t < t1 ? partials[t * kStatVals + k0] : fix_zero();
    }
#pragma unroll
    for (int u = 0; u < kAhead; ++u) acc = fix_add(acc, v[u]);
    if (clear) {
#pragma unroll
      for (int u = 0; u < kAhead; ++u) {
        const int t = tb + u * kWave;
        if (t < t1) partials[t * kStatVals + k0] = fix_zero();
      }
    }
  }
  acc = wave_sum_fix(acc);
  __shared__ Fix tot[kStatVals];
  if (lane == 0) tot[k0] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    Fix f[kStatVals];
    for (int k = 0; k < kStatVals; ++k) f[k] = tot[k];
    const bool bad = f[kStatBad].lo != 0ull || f[kStatBad].hi != 0ll;
    double v[9];
    for (int k = 0; k < 9; ++k) v[k] = bad ? __builtin_nan("") : fix_to_double(f[k]);
    double o[kRecLen];
    o[0] = v[0];
    o[1] = v[1];
    o[2] = v[2];
    o[3] = v[0] + v[1] + v[2];
    o[4] = v[3];
    o[5] = v[4];
    o[6] = v[5];
    o[7] = 2.0 * v[1] / (3.0 * (N - 1.0));
    o[8] = N / v[6];
    o[9] = (double)(now.step + (uint64_t)advance);
    o[10] = v[7];
    o[11] = v[8];
    double* hrow = nullptr;
    if (advance) hrow = hist + ((now.hist % hist_cap) * nrep + r) * kRecLen;
    for (int k = 0; k < kRecLen; ++k) {
      rec[r * kRecLen + k] = o[k];
      if (hrow) hrow[k] = o[k];
    }
    if (finish) {
      // one replica: this block is the last one, and the end of the kernel
      // publishes its writes (no device-wide fence needed)
      if (gridDim.x > 1u) __threadfence();
      if (gridDim.x == 1u || atomicAdd(ticket, 1u) == gridDim.x - 1u) {
        if (gridDim.x > 1u) __threadfence();
        step_end(now, d_step, d_hist_count, ctl, next, builds, advance);
        atomicExch(ticket, 0u);
      }
    }
  }
}

// Projection on the internal energies (Sec. 4.2): eps_i <- eps_i - (E - E0)/N
// per replica, E from the record of the unconstrained update, then the new
// 1/T_i when the EOS is evaluated inline.
template <bool BATCH>
__global__ void k_project(PState s, int64_t n, const Geo* __restrict__ geo, Phys P,
                          const double* __restrict__ rec, const double* __restrict__ E0,
                          int eos_inline, uint32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (status_set(status)) return;
  const uint32_t r = BATCH ? s.r[i].rep : 0u;
  const double shift = (rec[r * kRecLen + 3] - E0[r]) / (double)geo[r].n;
  const double e = s.eps[i] - shift;
  s.eps[i] = e;
  if (!(e > 0.0)) {
    atomicOr(status, ST_NEG_EINT);
  } else if (eos_inline) {
    s.r[i].invT = inv_temperature(P, e, status);
  }
}

// Target energy of the projection: the energy in the current record.
__global__ void k_capture_e0(const double* __restrict__ rec, double* __restrict__ E0, int nrep) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrep) E0[r] = rec[r * kRecLen + 3];
}

// ---------------------------------------------------------------------------
// Test hooks.
// ---------------------------------------------------------------------------
__global__ void k_debug_cells(PState s, int64_t n, const Geo* __restrict__ geo, int32_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Rec& rc = s.r[i];
  const Geo& g = geo[rc.rep];
  const int cx = cell_coord(rc.qx, g.scale[0], g.nc[0]);
  const int cy = cell_coord(rc.qy, g.scale[1], g.nc[1]);
  const int cz = cell_coord(rc.qz, g.scale[2], g.nc[2]);
  out[g.first + rc.id] = cx + g.nc[0] * (cy + g.nc[1] * cz);
}

// The identifier row (replica's first row + ID) of the particle in every
// memory slot.
__global__ void k_debug_order(PState s, int64_t n, const Geo* __restrict__ geo, int32_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Rec& rc = s.r[i];
  out[i] = (int32_t)(geo[rc.rep].first + rc.id);
}

// Every pair of the lists once, as (lower id, higher id) rows.  A pair
// joining two tiles is in both lists (taken from the lower identifier); with
// the tile work lists (uniq) a pair inside a tile is in one list only.
__global__ void k_debug_pairs(PState s, NList nl, int64_t n, const Geo* __restrict__ geo,
                              int uniq, int32_t* out, int64_t cap,
                              unsigned long long* counter) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Rec& a = s.r[i];
  const Geo& g = geo[a.rep];
  for (uint32_t k = 0; k < nl.count[i]; ++k) {
    const uint32_t j = nl.idx[(int64_t)k * nl.stride + i];
    const uint32_t idj = s.r[j].id;
    const bool once = uniq && (((uint32_t)i ^ j) < (uint32_t)kUniqTile);
    if (once || a.id < idj) {
      const unsigned long long slot = atomicAdd(counter, 1ull);
      if ((int64_t)slot < cap) {
        out[2 * slot] = (int32_t)(g.first + (a.id < idj ? a.id : idj));
        out[2 * slot + 1] = (int32_t)(g.first + (a.id < idj ? idj : a.id));
      }
    }
  }
}

__global__ void k_debug_rng(uint32_t key0, uint32_t key1, uint64_t step,
                            const uint32_t* __restrict__ lo, const uint32_t* __restrict__ hi,
                            int64_t n, uint32_t* raw, double* g, float* g32) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  Geo geo;
  geo.key0 = key0;
  geo.key1 = key1;
  uint32_t w[4];
  pair_words(geo, lo[k], hi[k], step, w);
  if (raw)
    for (int c = 0; c < 4; ++c) raw[4 * k + c] = w[c];
  if (g) {
    double G[3];
    box_muller_f64(w, G);
    for (int c = 0; c < 3; ++c) g[3 * k + c] = G[c];
  }
  if (g32) {
    float G[3];
    box_muller_f32(w, G);
    for (int c = 0; c < 3; ++c) g32[3 * k + c] = G[c];
  }
}

}  // namespace dpde
