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
// dissipation step), bucket histogram and ticket, identifier for the
// per-domain sort.
template <bool BATCH>
__global__ void k_dom_key(PState s, int64_t n, const Geo* __restrict__ geo,
                          uint32_t* __restrict__ dom, uint32_t* __restrict__ key,
                          uint32_t* __restrict__ ticket, uint32_t* __restrict__ idk,
                          uint32_t* __restrict__ count, const uint32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (status_set(status)) return;
  const Rec& rc = s.r[i];
  const Geo& g = geo[BATCH ? rc.rep : 0u];
  const uint32_t d = domain_index(g, rc.qx, rc.qy, rc.qz);
  dom[i] = d;
  key[i] = d;
  idk[i] = rc.id;
  ticket[i] = atomicAdd(&count[d], 1u);
}

// One lane per domain: its particles in increasing identifier order, each
// with its (identifier-sorted) neighbours of higher identifier in the same
// domain, i.e. the intra-domain pairs in increasing (lo, hi) order; every
// pair gets the exact Ornstein-Uhlenbeck step of its relative momentum at
// fixed gamma_ij (a = +(2 gamma_ij/m) chi dt), the internal energies share
// the kinetic-energy change, and finally 1/T of the domain's particles is
// refreshed for the SER sweeps.  Domains are disjoint, so no two lanes touch
// the same particle.
template <bool BATCH>
__global__ void k_ssa(PState s, NList nl, const uint32_t* __restrict__ dperm,
                      const uint32_t* __restrict__ dstart, int64_t ndoms,
                      const uint32_t* __restrict__ dom, const Geo* __restrict__ geo, Phys P,
                      const uint64_t* __restrict__ d_step, uint32_t* status) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= ndoms) return;
  if (status_set(status)) return;
  const uint64_t step = *d_step;
  Rec* R = s.r;
  double* eps = s.eps;
  const uint32_t b = dstart[d], e = dstart[d + 1];
  for (uint32_t k = b; k < e; ++k) {
    const uint32_t i = dperm[k];
    const uint32_t nn = nl.count[i];
    for (uint32_t m = 0; m < nn; ++m) {
      const uint32_t j = nl.idx[(int64_t)m * nl.stride + i];
      if (dom[j] != (uint32_t)d || R[j].id < R[i].id) continue;
      const Geo& g = geo[BATCH ? R[i].rep : 0u];
      const double ei = eps[i], ej = eps[j];
      if (!(ei > 0.0) || !(ej > 0.0)) {
        atomicOr(status, ST_NEG_EINT);
        return;
      }
      const double invT = inv_temperature(P, ei, status) + inv_temperature(P, ej, status);
      double dx, dy, dz;
      separation(g, R[i].qx, R[i].qy, R[i].qz, R[j].qx, R[j].qy, R[j].qz, dx, dy, dz);
      const double r2 = dist2(dx, dy, dz);
      const double r = r2 * inv_sqrt_f64(r2);
      const double w = 1.0 - r * P.inv_rc;
      const double chi = w * w;
      const double gij = P.gkT_half * invT;
      const double a = 2.0 * gij * P.inv_mass * chi * P.dt;
      const double decay = expm1(-a);
      const double var = gij > 0.0 ? -expm1(-2.0 * a) / gij : 4.0 * chi * P.dt * P.inv_mass;
      const double amp = P.sigma * sqrt(P.mass * var);
      uint32_t wd[4];
      pair_words(g, R[i].id, R[j].id, step, wd);  // i is the lower identifier
      double G[3];
      box_muller_f64(wd, G);
      const double pi[3] = {R[i].px, R[i].py, R[i].pz};
      const double pj[3] = {R[j].px, R[j].py, R[j].pz};
      double ni[3], nj[3], k0 = 0.0, k1 = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double D = decay * (pi[c] - pj[c]) + amp * G[c];
        ni[c] = pi[c] + 0.5 * D;
        nj[c] = pj[c] - 0.5 * D;
        k0 += pi[c] * pi[c] + pj[c] * pj[c];
        k1 += ni[c] * ni[c] + nj[c] * nj[c];
      }
      R[i].px = ni[0]; R[i].py = ni[1]; R[i].pz = ni[2];
      R[j].px = nj[0]; R[j].py = nj[1]; R[j].pz = nj[2];
      const double dK = (k1 - k0) * P.inv_2m;
      eps[i] = ei - 0.5 * dK;
      eps[j] = ej - 0.5 * dK;
    }
  }
  for (uint32_t k = b; k < e; ++k) {
    const uint32_t i = dperm[k];
    const double ei = eps[i];
    if (!(ei > 0.0)) {
      atomicOr(status, ST_NEG_EINT);
      return;
    }
    R[i].invT = inv_temperature(P, ei, status);
  }
}

}  // namespace dpde
