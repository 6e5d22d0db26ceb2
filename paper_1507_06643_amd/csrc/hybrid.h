// Hybrid scheme (Sec. 3.2.2): SSA (Sec. 3.1.2, eq. SSA_ij) for the pairs
// inside one spatial domain, SER for the pairs across domains.
#pragma once
#include "pairs.h"

namespace dpde {

// Domain of a position: ndom[d] equal slabs per dimension, clamped to the box
// (free boundaries can leave particles outside it).
__device__ __forceinline__ uint32_t domain_index(const Geo& g, double x, double y, double z) {
  const double q[3] = {x, y, z};
  int64_t c[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double v = floor(q[d] * g.dscale[d]);
    v = v < 0.0 ? 0.0 : v;
    v = v > (double)(g.ndom[d] - 1) ? (double)(g.ndom[d] - 1) : v;
    c[d] = (int64_t)v;
  }
  return (uint32_t)(g.dom_base + c[0] + (int64_t)g.ndom[0] * (c[1] + (int64_t)g.ndom[1] * c[2]));
}

// Domain of every particle (positions at the start of the fluctuation/
// dissipation step), bucket histogram and ticket (one atomic per run of
// equal domains in a wave), identifier for the per-domain ranking.
template <bool BATCH>
__global__ void k_dom_key(PState s, int64_t n, const Geo* __restrict__ geo,
                          uint32_t* __restrict__ dom, uint32_t* __restrict__ key,
                          uint32_t* __restrict__ ticket, uint32_t* __restrict__ idk,
                          uint32_t* __restrict__ count, const uint32_t* status) {
  if (status_set(status)) return;  // uniform
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < n;
  uint32_t d = 0xFFFFFFFFu;
  if (live) {
    const Rec& rc = s.r[i];
    const Geo& g = geo[BATCH ? rc.rep : 0u];
    d = domain_index(g, rc.qx, rc.qy, rc.qz);
    dom[i] = d;
    key[i] = d;
    idk[i] = rc.id;
  }
  const uint32_t t = run_ticket(d, live, count);
  if (live) ticket[i] = t;
}

// Rank of every particle inside its domain by identifier (the order the SSA
// sweep takes the domain's particles), out of place: one thread per bucket
// slot counts the smaller identifiers of its bucket.  lslot[i] is the rank.
// The thread also counts the particle's pairs of the sweep (below) for its
// sorted slot.
//
// The intra-domain pairs in the order of the SSA sweep: the domain's
// particles by increasing identifier, each with its list neighbours (in
// identifier order) of higher identifier in the same domain.  After a scan
// of the counts, k_ssa_pairs writes each pair's local slots, its weight
// chi = w(r)^2 and its noise G_ij (positions are fixed during the sweep, so
// both are known before it starts).
__global__ void k_dom_rank(const uint32_t* __restrict__ bucket, const uint32_t* __restrict__ dstart,
                           const uint32_t* __restrict__ dom, const uint32_t* __restrict__ idk,
                           int64_t n, NList nl, uint32_t* __restrict__ sorted,
                           uint32_t* __restrict__ lslot, uint32_t* __restrict__ pcnt,
                           const uint32_t* status) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  if (status_set(status)) return;
  const uint32_t i = bucket[k];
  const uint32_t d = dom[i];
  const uint32_t b = dstart[d], e = dstart[d + 1];
  const uint32_t my = idk[i];
  uint32_t r = 0;
  for (uint32_t m = b; m < e; ++m) r += idk[bucket[m]] < my ? 1u : 0u;
  sorted[b + r] = i;
  lslot[i] = r;
  uint32_t c = 0;
  const uint32_t nn = nl.count[i];
  for (uint32_t m = 0; m < nn; ++m) {
    const uint32_t j = nl.idx[(int64_t)m * nl.stride + i];
    c += (dom[j] == d && idk[j] > my) ? 1u : 0u;
  }
  pcnt[b + r] = c;
}

struct SsaPairs {
  uint2* idx;   // local slots (lower identifier first)
  Vec4* gc;     // G_ij in x, y, z and chi in w
  int64_t cap;
};

// One lane group per sorted slot: the group's lanes test the list entries
// in turn, and the pairs found in a trip take consecutive places in list order.
template <bool BATCH>
__global__ __launch_bounds__(kPairBlockMax) void k_ssa_pairs(
    PState s, NList nl, const uint32_t* __restrict__ sorted, const uint32_t* __restrict__ lslot,
    int64_t n, const uint32_t* __restrict__ dom, const uint32_t* __restrict__ idk,
    const uint32_t* __restrict__ poff, const Geo* __restrict__ geo, Phys P,
    const uint64_t* __restrict__ d_step, SsaPairs sp, uint32_t* status) {
  const Lanes L = lanes();
  if (L.i >= n) return;  // uniform in the group
  if (status_set(status)) return;
  const int64_t k = L.i;
  const uint64_t step = *d_step;
  const Rec* __restrict__ R = s.r;
  const uint32_t i = sorted[k];
  const uint32_t d = dom[i], id = idk[i], li = lslot[i];
  const double xi = R[i].qx, yi = R[i].qy, zi = R[i].qz;
  const Geo& g = geo[BATCH ? R[i].rep : 0u];
  const uint32_t nn = nl.count[i];
  int64_t t = poff[k];
  for (uint32_t base = 0; base < nn; base += kSub) {
    const uint32_t m = base + L.sub;
    uint32_t j = 0;
    bool take = false;
    if (m < nn) {
      j = nl.idx[(int64_t)m * nl.stride + i];
      take = dom[j] == d && idk[j] > id;  // the same test as k_dom_rank
    }
    const uint32_t bits = group_ballot(L, take);
    if (take) {
      const int64_t tt = t + __popc(bits & ((1u << L.sub) - 1u));
      if (tt >= sp.cap) {
        atomicOr(status, ST_OVERFLOW);
      } else {
        double dx, dy, dz;
        separation(g, xi, yi, zi, R[j].qx, R[j].qy, R[j].qz, dx, dy, dz);
        const double r2 = dist2(dx, dy, dz);
        const double r = r2 * inv_sqrt_f64(r2);
        const double w = 1.0 - r * P.inv_rc;
        uint32_t wd[4];
        pair_words(g, id, idk[j], step, wd);  // i is the lower identifier
        double G[3];
        box_muller_f64(wd, G);
        sp.idx[tt] = make_uint2(li, lslot[j]);
        sp.gc[tt] = Vec4{G[0], G[1], G[2], w * w};
      }
    }
    t += __popc(bits);
  }
}

// Momenta and internal energies of one domain's particles, addressed by
// their slot in the domain: in the lane's LDS column, or (large domains) in
// the particle arrays.
struct SsaLds {
  double* base;  // slot s: p_x, p_y, p_z, eps at base[4 s .. 4 s + 3]
  __device__ double& p(uint32_t s, int c) const { return base[4 * s + c]; }
  __device__ double& e(uint32_t s) const { return base[4 * s + 3]; }
};
struct SsaGlobal {
  Rec* R;
  double* eps;
  const uint32_t* sorted;  // the domain's first sorted slot onwards
  __device__ double& p(uint32_t s, int c) const {
    Rec& r = R[sorted[s]];
    return c == 0 ? r.px : (c == 1 ? r.py : r.pz);
  }
  __device__ double& e(uint32_t s) const { return eps[sorted[s]]; }
};

// The sweep over one domain's pairs: each gets the exact Ornstein-Uhlenbeck
// step of its relative momentum at fixed gamma_ij (a = +(2 gamma_ij/m) chi
// dt), and the internal energies share the kinetic-energy change.
template <class St>
__device__ bool ssa_sweep(const St& S, int64_t t0, int64_t t1, const SsaPairs& sp, const Phys& P,
                          uint32_t* status) {
  // the pair data do not depend on the sweep's state: requested two pairs
  // ahead, their latency overlaps the arithmetic of the current pair
  uint2 pr1{}, pr2{};
  Vec4 gc1{}, gc2{};
  if (t0 < t1) {
    pr1 = sp.idx[t0];
    gc1 = sp.gc[t0];
  }
  if (t0 + 1 < t1) {
    pr2 = sp.idx[t0 + 1];
    gc2 = sp.gc[t0 + 1];
  }
  for (int64_t t = t0; t < t1; ++t) {
    const uint2 pr = pr1;
    const Vec4 gc = gc1;
    pr1 = pr2;
    gc1 = gc2;
    if (t + 2 < t1) {
      pr2 = sp.idx[t + 2];
      gc2 = sp.gc[t + 2];
    }
    const uint32_t li = pr.x, lj = pr.y;
    const double ei = S.e(li), ej = S.e(lj);
    if (!(ei > 0.0) || !(ej > 0.0)) {
      atomicOr(status, ST_NEG_EINT);
      return false;
    }
    const double invT = inv_temperature(P, ei, status) + inv_temperature(P, ej, status);
    const double chi = gc.w;
    const double gij = P.gkT_half * invT;
    const double a = 2.0 * gij * P.inv_mass * chi * P.dt;
    const double decay = expm1(-a);
    const double var = gij > 0.0 ? -expm1(-2.0 * a) / gij : 4.0 * chi * P.dt * P.inv_mass;
    const double amp = P.sigma * sqrt(P.mass * var);
    const double G[3] = {gc.x, gc.y, gc.z};
    const double pi[3] = {S.p(li, 0), S.p(li, 1), S.p(li, 2)};
    const double pj[3] = {S.p(lj, 0), S.p(lj, 1), S.p(lj, 2)};
    double ni[3], nj[3], k0 = 0.0, k1 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double D = decay * (pi[c] - pj[c]) + amp * G[c];
      ni[c] = pi[c] + 0.5 * D;
      nj[c] = pj[c] - 0.5 * D;
      k0 += pi[c] * pi[c] + pj[c] * pj[c];
      k1 += ni[c] * ni[c] + nj[c] * nj[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      S.p(li, c) = ni[c];
      S.p(lj, c) = nj[c];
    }
    const double dK = (k1 - k0) * P.inv_2m;
    S.e(li) = ei - 0.5 * dK;
    S.e(lj) = ej - 0.5 * dK;
  }
  return true;
}

// One lane per domain (Sec. 3.2.2: SSA inside the domain), its pairs taken
// in the order above.  The wave's domains share an LDS pool of POOL
// particle slots, handed out by a prefix sum of the domain sizes; a domain
// beyond the pool sweeps in the particle arrays.  Finally 1/T of the domain's
// particles is refreshed for the SER sweeps.  Domains are disjoint, so no two
// lanes touch the same particle.
// Pool sizes: the host takes the smallest that holds the wave's domains at
// 1.25 times the mean size (the largest, 80 KiB, leaves two blocks per CU).
constexpr int kSsaPoolMax = 2560;

template <int POOL>
__global__ __launch_bounds__(kWave) void k_ssa_walk(PState s, const uint32_t* __restrict__ sorted,
                                                   const uint32_t* __restrict__ dstart,
                                                   int64_t ndoms, const uint32_t* __restrict__ poff,
                                                   SsaPairs sp, Phys P, uint32_t* status) {
  __shared__ double pool[POOL * 4];
  const int64_t d = (int64_t)blockIdx.x * kWave + threadIdx.x;
  const bool live = d < ndoms;
  const uint32_t b = live ? dstart[d] : 0u;
  const uint32_t c = live ? dstart[d + 1] - b : 0u;
  // inclusive prefix sum of the sizes over the wave (one wave per block)
  uint32_t end = c;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t v = (uint32_t)__shfl_up((int)end, o, kWave);
    if ((int)threadIdx.x >= o) end += v;
  }
  if (!live) return;  // no barrier below
  if (status_set(status)) return;
  Rec* R = s.r;
  double* eps = s.eps;
  const int64_t t0 = poff[b], t1 = min((int64_t)poff[b + c], sp.cap);
  if (end <= (uint32_t)POOL) {
    const SsaLds S{pool + 4 * (end - c)};
    for (uint32_t q = 0; q < c; ++q) {
      const uint32_t i = sorted[b + q];
      S.p(q, 0) = R[i].px;
      S.p(q, 1) = R[i].py;
      S.p(q, 2) = R[i].pz;
      S.e(q) = eps[i];
    }
    if (!ssa_sweep(S, t0, t1, sp, P, status)) return;
    for (uint32_t q = 0; q < c; ++q) {
      const uint32_t i = sorted[b + q];
      const double ei = S.e(q);
      R[i].px = S.p(q, 0);
      R[i].py = S.p(q, 1);
      R[i].pz = S.p(q, 2);
      eps[i] = ei;
      if (!(ei > 0.0)) {
        atomicOr(status, ST_NEG_EINT);
        return;
      }
      R[i].invT = inv_temperature(P, ei, status);
    }
  } else {
    const SsaGlobal S{R, eps, sorted + b};
    if (!ssa_sweep(S, t0, t1, sp, P, status)) return;
    for (uint32_t q = 0; q < c; ++q) {
      const uint32_t i = sorted[b + q];
      const double ei = eps[i];
      if (!(ei > 0.0)) {
        atomicOr(status, ST_NEG_EINT);
        return;
      }
      R[i].invT = inv_temperature(P, ei, status);
    }
  }
}

}  // namespace dpde
