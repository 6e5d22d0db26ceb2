// Particle storage and cell binning.
//
// Storage: one 64-byte record per particle (position, momentum, 1/T, id,
// replica), so that gathering a neighbour touches one cache line instead of
// one line per array; the internal energy, read only by its own particle,
// lives in a separate array.
//
// Order: particles are kept sorted by the composite key (cell, id).  The sort
// is a two-level MSD radix sort: digit 1 is the whole cell index (one
// counting pass: histogram of cells with integer atomics, exclusive scan to
// cell offsets, scatter by offset + arrival ticket); digit 2 is the particle
// identifier, finished inside each cell bucket by insertion sort (buckets
// hold ~3 particles at density 3 with cells of side ~rc).  The resulting order
// is a pure function of the positions, independent of the previous order and
// of atomic arrival order, so trajectories are bit reproducible and a resumed
// run continues exactly.
#pragma once

#include "common.h"

namespace dpde {

struct alignas(64) Rec {
  double qx, qy, qz;
  double px, py, pz;
  double invT;
  uint32_t id;   // identifier inside the replica
  uint32_t rep;  // replica index
};
static_assert(sizeof(Rec) == 64, "particle record must be one 64-byte block");

struct PState {
  Rec* r;
  double* eps;
};

// Neighbour-list build control for one step.  The kick kernel raises dmax to
// the largest squared displacement since the last build (bit pattern of a
// non-negative double, so integer max is float max); the binning and list
// build kernels run when force is set or dmax exceeds (skin/2)^2, and do
// nothing otherwise.  The decision is read from device memory by every
// kernel, so a captured graph replays it faithfully.
struct BuildCtl {
  unsigned long long dmax_bits;
  uint32_t force;
  uint32_t pad;
  unsigned long long qmax_bits;  // largest |coordinate| outside the box this step
};

__device__ __forceinline__ bool rebuild_now(const BuildCtl* c, double half_skin2) {
  return c->force != 0u || __longlong_as_double((long long)c->dmax_bits) > half_skin2;
}

// Position (FP32) and identifier of a particle in 16 bytes: what the list
// build's candidate scans read (written by the reorder), and the reference
// of the kick's displacement test until the next build.  The FP32 distance
// test is widened by a bound on its rounding error, so a list still holds
// every pair within rc + skin; the exact r < rc filter of each step is FP64.
struct alignas(16) QIdF {
  float x, y, z;
  uint32_t id;
};

// XCD-aware tile order: the hardware deals workgroups round-robin over the 8
// XCDs (each with its own L2); the remap makes XCD x work through one
// contiguous share of the cell-sorted particles, a slab of the box whose
// neighbour data stays in that XCD's L2.  It is a bijection on [0, nb).
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nb) {
  constexpr unsigned kXcd = 8;
  const unsigned q = nb / kXcd, r = nb % kXcd;
  const unsigned x = b % kXcd, k = b / kXcd;
  // workgroups b = x + 8k with k < q + (x < r) land on XCD x; give them the
  // consecutive tiles first(x) .. first(x) + q + (x < r) - 1
  const unsigned first = x * q + (x < r ? x : r);
  return first + k;
}

// ---- initial load: AoS rows in identifier order -> records --------------------
// Row k belongs to the replica r with geo[r].first <= k < geo[r].first + n.
__global__ void k_load_state(const double* __restrict__ q, const double* __restrict__ p,
                             const double* __restrict__ eps, const Geo* __restrict__ geo, int nrep,
                             int64_t n, PState s, uint32_t* status) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int lo = 0, hi = nrep - 1;
  while (lo < hi) {  // last replica whose first row <= k
    const int mid = (lo + hi + 1) >> 1;
    if (geo[mid].first <= k) lo = mid; else hi = mid - 1;
  }
  Rec rc;
  rc.qx = q[3 * k]; rc.qy = q[3 * k + 1]; rc.qz = q[3 * k + 2];
  rc.px = p[3 * k]; rc.py = p[3 * k + 1]; rc.pz = p[3 * k + 2];
  rc.invT = 0.0;
  rc.id = (uint32_t)(k - geo[lo].first);
  rc.rep = (uint32_t)lo;
  const double e = eps[k];
  s.r[k] = rc;
  s.eps[k] = e;
  const bool fin = isfinite(rc.qx) && isfinite(rc.qy) && isfinite(rc.qz) && isfinite(rc.px) &&
                   isfinite(rc.py) && isfinite(rc.pz) && isfinite(e);
  if (!fin) atomicOr(status, ST_NONFINITE);
  else if (!(e > 0.0)) atomicOr(status, ST_NEG_EINT);
}

// ---- state out: records -> AoS rows in identifier order -----------------------
__global__ void k_store_state(PState s, const Geo* __restrict__ geo, int64_t n, double* q,
                              double* p, double* eps) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Rec rc = s.r[i];
  const int64_t row = geo[rc.rep].first + (int64_t)rc.id;
  if (q) { q[3 * row] = rc.qx; q[3 * row + 1] = rc.qy; q[3 * row + 2] = rc.qz; }
  if (p) { p[3 * row] = rc.px; p[3 * row + 1] = rc.py; p[3 * row + 2] = rc.pz; }
  if (eps) eps[row] = s.eps[i];
}

__global__ void k_store_vec3(PState s, const Geo* __restrict__ geo, int64_t n,
                             const double* __restrict__ x, const double* __restrict__ y,
                             const double* __restrict__ z, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Rec& rc = s.r[i];
  const int64_t row = geo[rc.rep].first + (int64_t)rc.id;
  out[3 * row] = x[i]; out[3 * row + 1] = y[i]; out[3 * row + 2] = z[i];
}

// 1/T_i of every particle into out (identifier order).
__global__ void k_store_inv_temperature(PState s, const Geo* __restrict__ geo, int64_t n,
                                        double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Rec& rc = s.r[i];
  out[geo[rc.rep].first + (int64_t)rc.id] = rc.invT;
}

// Length of every particle's list of the step into out (identifier order).
__global__ void k_store_list_length(PState s, const Geo* __restrict__ geo, int64_t n,
                                    const uint32_t* __restrict__ count, int32_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Rec& rc = s.r[i];
  out[geo[rc.rep].first + (int64_t)rc.id] = (int32_t)count[i];
}

constexpr int kAuxMaxThreads = 1024;  // largest block of the per-particle kernels

// First half of velocity-Verlet (Sec. 3.1) on one record: p += dt/2 F and
// q += dt p / m (kick != 0), then the periodic wrap into [0, L).  Returns in
// d2 the square of an upper bound on the displacement since the last list
// build and, for a coordinate outside [0, box) (free boundaries), the
// largest such |q| in qa; a non-finite p or q raises the status.  The one
// definition of this arithmetic: k_kick and the end of the tile sweep 2
// both call it.
__device__ __forceinline__ void kick_record(Rec& rc, const double F[3], const Geo& g,
                                            const Phys& P, int kick,
                                            const QIdF* __restrict__ ref, int64_t i,
                                            double& d2, double& qa, uint32_t* status) {
  double q[3] = {rc.qx, rc.qy, rc.qz};
  if (kick) {
    double p[3] = {rc.px, rc.py, rc.pz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      p[d] = p[d] + P.half_dt * F[d];
      q[d] = q[d] + P.dt * p[d] / P.mass;
    }
    rc.px = p[0]; rc.py = p[1]; rc.pz = p[2];
    if (!(isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]))) atomicOr(status, ST_NONFINITE);
  }
#pragma unroll
  for (int d = 0; d < 3; ++d)
    if (g.periodic[d]) q[d] = wrap_coord(q[d], g.box[d]);
  rc.qx = q[0]; rc.qy = q[1]; rc.qz = q[2];
  if (!(isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2]))) {
    atomicOr(status, ST_NONFINITE);
  } else {
    // coordinates outside [0, box) (free boundaries) for the list build's
    // rounding margin; inside, the box side bounds them already
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (!(q[d] >= 0.0 && q[d] < g.box[d])) qa = fmax(qa, fabs(q[d]));
    // The reference is the build-time position rounded to FP32, each
    // coordinate within 2^-24 |x| of the exact one, which is below
    // 2^-23 |x_f| for its FP32 value x_f (2^-149 covers subnormals); the sum
    // of those bounds and 2^-50 of the FP64 distance for its own rounding
    // make d an upper bound on the true displacement.
    const QIdF r0 = ref[i];
    double dx = q[0] - (double)r0.x, dy = q[1] - (double)r0.y, dz = q[2] - (double)r0.z;
    if (g.periodic[0]) dx = min_image(dx, g.box[0], g.half_box[0]);
    if (g.periodic[1]) dy = min_image(dy, g.box[1], g.half_box[1]);
    if (g.periodic[2]) dz = min_image(dz, g.box[2], g.half_box[2]);
    const double slack =
        0x1p-23 * ((double)fabsf(r0.x) + (double)fabsf(r0.y) + (double)fabsf(r0.z)) + 0x1p-147;
    const double d = sqrt(dx * dx + dy * dy + dz * dz) * (1.0 + 0x1p-50) + slack;
    d2 = d * d;
  }
}

// Raise a running maximum of non-negative doubles kept as bits (they order
// like their bit patterns); one atomic, and only when it raises the value (a
// stale read can only be smaller than the true value, never skip a raise).
__device__ __forceinline__ void raise_max_bits(unsigned long long* where, double v) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
  const unsigned long long cur = __hip_atomic_load(where, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (bits > cur) atomicMax(where, bits);
}

// The kick of every particle (kick == 0: only the wrap), with the maxima the
// next list-build decision reads.
template <bool BATCH>
__global__ void k_kick(PState s, const double* __restrict__ Fx, const double* __restrict__ Fy,
                       const double* __restrict__ Fz, int64_t n, const Geo* __restrict__ geo,
                       Phys P, int kick, const QIdF* __restrict__ ref, BuildCtl* ctl,
                       uint32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // no early return: every thread reaches the block barrier below (another
  // block may raise the status while this one runs)
  const bool run = !status_set(status);
  double d2 = 0.0, qa = 0.0;
  if (run && i < n) {
    Rec rc = s.r[i];
    const Geo& g = geo[BATCH ? rc.rep : 0u];
    double F[3] = {0.0, 0.0, 0.0};
    if (kick) {
      F[0] = Fx[i];
      F[1] = Fy[i];
      F[2] = Fz[i];
    }
    kick_record(rc, F, g, P, kick, ref, i, d2, qa, status);
    s.r[i] = rc;
  }
  // |q| outside the box only occurs with free boundaries: waves that have
  // any take their maximum and one atomic (when it raises the running one)
  if (__any(qa > 0.0)) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) qa = fmax(qa, __shfl_xor(qa, off, kWave));
    if ((threadIdx.x % kWave) == 0 && run) raise_max_bits(&ctl->qmax_bits, qa);
  }
  // block maximum of the displacement, then one atomic per block
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) d2 = fmax(d2, __shfl_xor(d2, off, kWave));
  __shared__ double wmax[kAuxMaxThreads / kWave];
  const int nw = blockDim.x / kWave;
  if ((threadIdx.x % kWave) == 0) wmax[threadIdx.x / kWave] = d2;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < nw; ++w) d2 = fmax(d2, wmax[w]);
    if (run) raise_max_bits(&ctl->dmax_bits, d2);
  }
}

// Histogram increment with one atomic per run of equal keys among
// consecutive lanes of a wave; the run's lanes take consecutive tickets.
// Every lane of the wave calls (dead lanes with live = false).
__device__ __forceinline__ uint32_t run_ticket(uint32_t c, bool live, uint32_t* count) {
  const int lane = threadIdx.x % kWave;
  const uint32_t prev = __shfl_up(c, 1, kWave);
  const bool head = live && (lane == 0 || prev != c);
  const unsigned long long heads = __ballot(head);
  const unsigned long long below = (lane == 63) ? ~0ull : ((1ull << (lane + 1)) - 1ull);
  const int my_head = 63 - __clzll(heads & below);  // last head at or below this lane
  const unsigned long long above = heads & ~below;   // heads strictly above
  const int next_head = above ? __ffsll((long long)above) - 1 : kWave;
  // the run of a head ends before the next head or at the first dead lane
  const unsigned long long alive = __ballot(live);
  int run_end = next_head;
  const unsigned long long dead_above = ~alive & ~below;
  if (dead_above) {
    const int first_dead = __ffsll((long long)dead_above) - 1;
    if (first_dead < run_end) run_end = first_dead;
  }
  uint32_t base = 0;
  if (head) base = atomicAdd(&count[c], (uint32_t)(run_end - lane));
  base = __shfl(base, my_head, kWave);
  return base + (uint32_t)(lane - my_head);
}

// Cell key of every particle and the cell histogram (list-build steps only).
// The identifier is also written to a compact array for the per-cell sort.
// The histogram update is aggregated per run of equal keys inside a wave (the
// particles are still nearly in cell order): one atomic per run, the run's
// lanes take consecutive tickets.  Tiles follow the XCD-aware order, so each
// XCD's atomics touch its own slab of counters.
template <bool BATCH>
__global__ void k_bin_key(PState s, int64_t n, const Geo* __restrict__ geo,
                          uint32_t* __restrict__ key, uint32_t* __restrict__ ticket,
                          uint32_t* __restrict__ idk, uint32_t* __restrict__ count,
                          const BuildCtl* ctl, double half_skin2, uint32_t* status) {
  if (status_set(status) || !rebuild_now(ctl, half_skin2)) return;  // uniform
  const int64_t i = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const bool live = i < n;
  uint32_t c = 0xFFFFFFFFu;
  if (live) {
    const Rec& rc = s.r[i];
    const Geo& g = geo[BATCH ? rc.rep : 0u];
    const int cx = cell_coord(rc.qx, g.scale[0], g.nc[0]);
    const int cy = cell_coord(rc.qy, g.scale[1], g.nc[1]);
    const int cz = cell_coord(rc.qz, g.scale[2], g.nc[2]);
    c = (uint32_t)(g.cell_base + cell_key(g, cx, cy, cz));
    key[i] = c;
    idk[i] = rc.id;
  }
  const uint32_t t = run_ticket(c, live, count);
  if (live) ticket[i] = t;
}

// ---- exclusive scan of the cell histogram -> cell offsets --------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// Exclusive scan of one value per thread across the block; returns the block
// total through *total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* smem,
                                                         uint32_t* total) {
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  if (lane == kWave - 1) smem[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int w = 0; w < nw; ++w) {
      const uint32_t t = smem[w];
      smem[w] = run;
      run += t;
    }
    smem[nw] = run;
  }
  __syncthreads();
  const uint32_t excl = smem[wid] + x - v;
  *total = smem[nw];
  __syncthreads();
  return excl;
}

__global__ void k_scan_tiles(const uint32_t* __restrict__ in, int64_t n,
                             uint32_t* __restrict__ tile_sums, const BuildCtl* ctl,
                             double half_skin2) {
  if (!rebuild_now(ctl, half_skin2)) return;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) s += in[base + k];
  __shared__ uint32_t smem[kScanThreads / kWave + 1];
  uint32_t total;
  block_exclusive_scan(s, smem, &total);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// out[c] = sum_{c' < c} in[c'] for c <= n; the histogram is cleared for the
// next step.  Each block first adds the totals of the tiles before it (at
// most 1024 * 8 tiles: 32 per thread), so no separate pass scans them.
__global__ void k_scan_apply(uint32_t* __restrict__ in, int64_t n,
                             const uint32_t* __restrict__ tile_sums, uint32_t* __restrict__ out,
                             const BuildCtl* ctl, double half_skin2) {
  if (!rebuild_now(ctl, half_skin2)) return;
  __shared__ uint32_t smem[kScanThreads / kWave + 1];
  uint32_t before = 0;
  for (unsigned t = threadIdx.x; t < blockIdx.x; t += blockDim.x) before += tile_sums[t];
  uint32_t offset;
  block_exclusive_scan(before, smem, &offset);
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0u;
    s += v[k];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(s, smem, &total) + offset;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) {
      out[base + k] = run;
      in[base + k] = 0u;
    }
    run += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = offset + total;
}

// perm[offset[key] + ticket] = old slot.
__global__ void k_scatter(const uint32_t* __restrict__ key, const uint32_t* __restrict__ ticket,
                          const uint32_t* __restrict__ start, int64_t n,
                          uint32_t* __restrict__ perm, const BuildCtl* ctl, double half_skin2,
                          const uint32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (status_set(status) || !rebuild_now(ctl, half_skin2)) return;
  perm[start[key[i]] + ticket[i]] = (uint32_t)i;
}

// ---- digit 2 and the move into the new order (list-build steps) ------------
// One thread per bucket slot counts the smaller identifiers of its cell's
// bucket, which is its place in the cell, and writes its particle's record
// and internal energy there in the spare buffer, with the build-time position
// (FP32) and the memory index of the particle's identifier row (for the
// neighbour-list build).  The list build then returns the records to the
// working buffer, so the buffer roles never depend on whether this step
// rebuilt.
template <bool BATCH>
__global__ void k_rank_gather(PState src, PState dst, const uint32_t* __restrict__ bucket,
                              const uint32_t* __restrict__ start, const uint32_t* __restrict__ key,
                              const uint32_t* __restrict__ idk, int64_t n,
                              const Geo* __restrict__ geo, QIdF* __restrict__ qid,
                              uint32_t* __restrict__ slot, const BuildCtl* ctl, double half_skin2,
                              const uint32_t* status) {
  if (status_set(status) || !rebuild_now(ctl, half_skin2)) return;  // uniform
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = k < n;
  uint32_t i = 0, b = 0, e = 0, my = 0;
  if (live) {
    i = bucket[k];
    const uint32_t c = key[i];
    b = start[c];
    e = start[c + 1];
    my = idk[i];
  }
  // A cell's members hold consecutive slots, so a cell that lies within the
  // wave's 64 slots finds its members' identifiers on the other lanes; a
  // cell that crosses the wave's ends reads them from memory.
  const int lane = (int)(threadIdx.x % kWave);
  const int64_t w0 = k - lane;  // the wave's first slot
  const bool inwave = live && (int64_t)b >= w0 && (int64_t)e <= w0 + kWave;
  const uint32_t span = inwave ? e - b : 0u;
  uint32_t smax = span;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1)
    smax = max(smax, (uint32_t)__shfl_xor((int)smax, off, kWave));
  smax = (uint32_t)__builtin_amdgcn_readfirstlane((int)smax);
  uint32_t r = 0;
  for (uint32_t t = 0; t < smax; ++t) {  // every lane takes part in each read
    const int from = t < span ? (int)((int64_t)b - w0) + (int)t : lane;
    const uint32_t o = (uint32_t)__shfl((int)my, from, kWave);
    r += (t < span && o < my) ? 1u : 0u;
  }
  if (!live) return;
  if (!inwave)
    for (uint32_t m = b; m < e; ++m) r += idk[bucket[m]] < my ? 1u : 0u;
  const uint32_t p = b + r;
  const Rec rc = src.r[i];
  dst.r[p] = rc;
  dst.eps[p] = src.eps[i];
  qid[p] = QIdF{(float)rc.qx, (float)rc.qy, (float)rc.qz, rc.id};
  slot[(BATCH ? (uint32_t)geo[rc.rep].first : 0u) + rc.id] = p;
}

}  // namespace dpde
