// libdpde.so: host side of the C ABI declared in include/dpde.h.
//
// One handle = one or more systems (replicas) stored back to back in
// structure-of-arrays form, sorted by (replica, cell, id).  A step is a fixed
// sequence of kernel launches on the handle's stream; the host only reads the
// device status word once per dpde_step call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dpde.h"
#include "bin.h"
#include "mlp.h"
#include "pairs.h"
#include "hybrid.h"

using namespace dpde;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(DPDE_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                              \
  } while (0)

constexpr int kHistBytes = 64 << 20;
constexpr int kOrderBlockMax = 8;  // largest edge of the cell blocks of the memory order
constexpr int64_t kStatTile = 2048;

struct ProfileRec {
  const char* name;
  hipEvent_t a, b;
};

}  // namespace

struct dpde_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t user_stream = nullptr;
  Phys phys{};
  int nrep = 1;
  bool batch = false;
  std::vector<Geo> geo_h;
  std::vector<int64_t> offsets;
  Geo* geo = nullptr;
  int64_t n = 0;
  int64_t ncells = 0;
  int64_t step = 0;
  int pair_block = 256;
  int aux_block = 256;
  // SER sweeps with a pair inside a 128-particle tile evaluated once
  // (k_pass_b_uniq, k_pass_c_uniq) rather than every pair term on both
  // particles' lanes (k_pass_b, k_pass_c)
  bool pairs_once = true;

  PState cur{}, alt{};
  double half_skin2 = 0.0, rs2 = 0.0;
  QIdF* qid = nullptr;  // build-time FP32 positions and identifiers, cell order
  double box_max = 0.0;  // largest box side over the replicas
  uint32_t* slot = nullptr;  // memory index of each identifier row
  BuildCtl* ctl = nullptr;
  BuildCtl* ctl_next = nullptr;  // maxima of a kick fused into the previous sweep 2
  unsigned long long* builds = nullptr;
  SkinList skin{};
  bool regen = false;  // regenerate the noise in sweep 2 instead of storing dp_ij
  double *Fx = nullptr, *Fy = nullptr, *Fz = nullptr;
  Vec4* dpi = nullptr;  // dp_i of SER sweep 1
  H3* hv = nullptr;   // (p_i + dp_i/2) / m
  double* deps = nullptr;
  uint32_t* idk = nullptr;
  double* Ui = nullptr;
  uint32_t *key = nullptr, *ticket = nullptr;
  uint32_t* bucket = nullptr;  // cell buckets in ticket order (before the ranking)
  uint32_t *cell_count = nullptr, *cell_start = nullptr, *scan_tmp = nullptr;
  int scan_tiles = 0;
  NList nl{};
  uint32_t* status = nullptr;
  uint64_t* d_step = nullptr;
  int64_t* d_hist_count = nullptr;
  int64_t* tile_begin = nullptr;
  int32_t* rep_tile0 = nullptr;
  int ntiles = 0;
  Fix* partials = nullptr;
  // observables' partial sums added by the tile sweep 2 into slots
  // (nslots_u per replica)
  Fix* partials_u = nullptr;
  int32_t* rep_tile0_u = nullptr;
  int nslots_u = 0;
  int64_t min_rep_n = 0;  // particles of the smallest replica
  double* E0 = nullptr;   // per-replica target energy of the projection
  double* Li = nullptr;   // per-particle Laplacian share of U
  // Hybrid: domain of each particle, domain order, bucket offsets
  bool hybrid = false;
  int64_t ndoms = 0;
  int dscan_tiles = 0;
  uint32_t* dom = nullptr;
  uint32_t* dbucket = nullptr;  // particles by domain, in ticket order
  uint32_t* dperm = nullptr;    // particles by domain, by identifier inside each
  uint32_t* lslot = nullptr;    // rank of a particle inside its domain
  uint32_t* dcount = nullptr;
  uint32_t* dstart = nullptr;
  uint32_t* dscan_tmp = nullptr;
  // intra-domain pairs in SSA order: count per sorted slot, offsets, pairs
  int pscan_tiles = 0;
  uint32_t* pcnt = nullptr;
  uint32_t* poff = nullptr;
  uint32_t* pscan_tmp = nullptr;
  SsaPairs ssa{};
  BuildCtl* always = nullptr;  // a build control that always says 'now'
  double* rec = nullptr;
  double* hist = nullptr;
  int64_t hist_cap = 0;
  unsigned long long* counter = nullptr;
  uint32_t* stats_ticket = nullptr;  // blocks of the observables' final pass done

  // surrogate network
  MlpState mlp{};

  // profiling
  bool profiling = false;
  std::vector<ProfileRec> prof;
  std::vector<hipEvent_t> event_pool;

  // graph cache
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  int64_t graph_steps = 0;
  PState graph_cur{}, graph_alt{};  // buffer layout the graph was captured with

  std::vector<void*> allocations;
};

namespace {

template <typename T>
int dalloc(dpde_handle* h, T** p, size_t count) {
  void* ptr = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(&ptr, count * sizeof(T));
  if (e != hipSuccess)
    return fail(DPDE_ENOMEM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T),
                hipGetErrorString(e));
  h->allocations.push_back(ptr);
  *p = reinterpret_cast<T*>(ptr);
  return DPDE_OK;
}

hipEvent_t get_event(dpde_handle* h) {
  if (!h->event_pool.empty()) {
    hipEvent_t e = h->event_pool.back();
    h->event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch with optional per-kernel event timing.
template <typename... KArgs, typename... Args>
void launch(dpde_handle* h, const char* name, void (*kernel)(KArgs...), dim3 grid, dim3 block,
            Args... args) {
  if (grid.x == 0) return;
  if (h->profiling) {
    ProfileRec r{name, get_event(h), get_event(h)};
    (void)hipEventRecord(r.a, h->stream);
    hipLaunchKernelGGL(kernel, grid, block, 0, h->stream, args...);
    (void)hipEventRecord(r.b, h->stream);
    h->prof.push_back(r);
  } else {
    hipLaunchKernelGGL(kernel, grid, block, 0, h->stream, args...);
  }
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

int check_params(const dpde_params* P, bool first) {
  if (!P) return fail(DPDE_EINVAL, "params is NULL");
  if (P->n < 2) return fail(DPDE_EINVAL, "n = %lld < 2", (long long)P->n);
  if (P->n >= (int64_t)1 << 31) return fail(DPDE_EINVAL, "n = %lld too large", (long long)P->n);
  for (int d = 0; d < 3; ++d) {
    if (!(std::isfinite(P->box[d]) && P->box[d] > 0))
      return fail(DPDE_EINVAL, "box[%d] must be finite and > 0", d);
    if (P->periodic[d] != 0 && P->periodic[d] != 1)
      return fail(DPDE_EINVAL, "periodic[%d] must be 0 or 1", d);
  }
  if (!first) return DPDE_OK;
  if (!(std::isfinite(P->rc) && P->rc > 0)) return fail(DPDE_EINVAL, "rc must be > 0");
  if (!(std::isfinite(P->mass) && P->mass > 0)) return fail(DPDE_EINVAL, "mass must be > 0");
  if (!(std::isfinite(P->dt) && P->dt > 0)) return fail(DPDE_EINVAL, "dt must be > 0");
  if (!(std::isfinite(P->kT_ref) && P->kT_ref > 0)) return fail(DPDE_EINVAL, "kT_ref must be > 0");
  if (!(std::isfinite(P->gamma) && P->gamma >= 0)) return fail(DPDE_EINVAL, "gamma must be >= 0");
  if (!(std::isfinite(P->a) && P->a >= 0)) return fail(DPDE_EINVAL, "a must be >= 0");
  if (!(std::isfinite(P->skin) && P->skin >= 0 && P->skin <= P->rc))
    return fail(DPDE_EINVAL, "skin must be in [0, rc]");
  if (P->eos == DPDE_EOS_LINEAR) {
    if (!(std::isfinite(P->cv) && P->cv > 0)) return fail(DPDE_EINVAL, "cv must be > 0");
  } else if (P->eos == DPDE_EOS_EINSTEIN) {
    if (!(P->eos_n >= 0 && P->eos_omega > 0 && P->eos_c0 > 0 && std::isfinite(P->eos_n) &&
          std::isfinite(P->eos_omega) && std::isfinite(P->eos_c0)))
      return fail(DPDE_EINVAL, "Einstein EOS needs eos_n >= 0, eos_omega > 0, eos_c0 > 0");
  } else {
    return fail(DPDE_EINVAL, "unknown eos %d", P->eos);
  }
  if (P->precision != DPDE_FP64 && P->precision != DPDE_FP32)
    return fail(DPDE_EINVAL, "unknown precision %d", P->precision);
  if (P->model != DPDE_MODEL_VECTOR && P->model != DPDE_MODEL_PROJECTED)
    return fail(DPDE_EINVAL, "unknown model %d", P->model);
  if (P->scheme == DPDE_SCHEME_HYBRID) {
    if (P->model != DPDE_MODEL_VECTOR)
      return fail(DPDE_EINVAL, "the Hybrid scheme is implemented for the vector model");
    if (P->flags & DPDE_FLAG_REGENERATE_NOISE)
      return fail(DPDE_EINVAL, "the Hybrid scheme stores the SER increments");
    for (int d = 0; d < 3; ++d)
      if (P->ndom[d] < 1 || P->ndom[d] > (1 << 20))
        return fail(DPDE_EINVAL, "ndom[%d] must be in [1, 2^20]", d);
  }
  if (P->potential == DPDE_POT_LJ) {
    if (!(std::isfinite(P->eps_lj) && P->eps_lj > 0 && std::isfinite(P->r_lj) && P->r_lj > 0))
      return fail(DPDE_EINVAL, "LJ needs eps_lj > 0 and r_lj > 0");
  } else if (P->potential != DPDE_POT_SOFT) {
    return fail(DPDE_EINVAL, "unknown potential %d", P->potential);
  }
  if ((P->flags & ~(DPDE_FLAG_REGENERATE_NOISE | DPDE_FLAG_PROJECT_EINT)) != 0)
    return fail(DPDE_EINVAL, "unknown flags 0x%x", P->flags);
  if (P->theta_mode < 0 || P->theta_mode > 2)
    return fail(DPDE_EINVAL, "unknown theta_mode %d", P->theta_mode);
  if (P->scheme != DPDE_SCHEME_SER && P->scheme != DPDE_SCHEME_SEM &&
      P->scheme != DPDE_SCHEME_HYBRID)
    return fail(DPDE_EINVAL, "unknown scheme %d", P->scheme);
  if (P->neighbor_cap < 0 || P->neighbor_cap > 1024)
    return fail(DPDE_EINVAL, "neighbor_cap must be in [0, 1024]");
  return DPDE_OK;
}

int geometry(const dpde_params* P, Geo& g) {
  for (int d = 0; d < 3; ++d) {
    const double ncd = std::floor(P->box[d] / (P->rc + P->skin));
    if (ncd < 3.0)
      return fail(DPDE_EBOX, "box[%d] = %g holds %g < 3 cells of side rc + skin = %g", d,
                  P->box[d], ncd, P->rc + P->skin);
    if (ncd > 1e6) return fail(DPDE_EINVAL, "box[%d]/rc too large", d);
    g.nc[d] = (int32_t)ncd;
    g.box[d] = P->box[d];
    g.half_box[d] = 0.5 * P->box[d];
    g.scale[d] = (double)g.nc[d] / P->box[d];
    g.periodic[d] = P->periodic[d];
  }
  g.oblk = 1;
  g.oblk_inv = 1.0f;
  g.key0 = (uint32_t)P->seed;
  g.key1 = (uint32_t)(P->seed >> 32) ^ P->replica;
  for (int d = 0; d < 3; ++d) {
    g.ndom[d] = P->scheme == DPDE_SCHEME_HYBRID ? P->ndom[d] : 1;
    g.dscale[d] = (double)g.ndom[d] / P->box[d];
  }
  return DPDE_OK;
}

void physics(const dpde_params* P, Phys& ph) {
  ph.mass = P->mass;
  ph.inv_mass = 1.0 / P->mass;
  ph.inv_2m = 1.0 / (2.0 * P->mass);
  ph.rc = P->rc;
  ph.inv_rc = 1.0 / P->rc;
  ph.rc2 = P->rc * P->rc;
  ph.a = P->a;
  ph.half_a_rc = 0.5 * P->a * P->rc;
  ph.gkT_half = 0.5 * P->gamma * P->kT_ref;
  ph.sigma = std::sqrt(2.0 * P->gamma * P->kT_ref);
  ph.dt = P->dt;
  ph.half_dt = 0.5 * P->dt;
  ph.sqrt_dt = std::sqrt(P->dt);
  // Ito term of the SEM energy update: one noise dimension per component of
  // G_ij (3), or the single scalar of the projected model (1)
  ph.dsigma2_m = (P->model == DPDE_MODEL_PROJECTED ? 1.0 : 3.0) * ph.sigma * ph.sigma / P->mass;
  ph.model = P->model;
  ph.potential = P->potential;
  ph.reach = P->rc + 2.0 * P->skin;
  ph.project = (P->flags & DPDE_FLAG_PROJECT_EINT) != 0;
  ph.lj4e = 4.0 * P->eps_lj;
  ph.r_lj2 = P->r_lj * P->r_lj;
  {
    // v_LJ(rc) and v_LJ'(rc) of the spline (eq. Ep: v(rc) = v'(rc) = 0)
    const double s6 = std::pow(P->r_lj / P->rc, 6.0);
    ph.lj_vc = 4.0 * P->eps_lj * (s6 * s6 - s6);
    ph.lj_dvc = -24.0 * P->eps_lj * (2.0 * s6 * s6 - s6) / P->rc;
  }
  ph.cv = P->cv;
  ph.eos_n = P->eos_n;
  ph.eos_omega = P->eos_omega;
  ph.eos_c0 = P->eos_c0;
  ph.eos = P->eos;
  ph.theta_mode = P->theta_mode;
  ph.precision = P->precision;
  ph.scheme = P->scheme;
  ph.cap = P->neighbor_cap > 0 ? P->neighbor_cap : (P->skin > 0 ? 96 : 64);
  // finest grid with a pair force a w r_hat (|.| <= a) and a potential share
  // a rc w^2 / 4 at least a factor 2 inside the range 2^(51-g)
  {
    const double bound = std::max(P->a, 0.25 * P->a * P->rc);
    int g = 46;
    while (g > 30 && !(2.0 * bound < std::ldexp(1.0, 51 - g))) --g;
    ph.fix_scale_f = std::ldexp(1.0, g);
    ph.fix_inv_f = std::ldexp(1.0, -g);
    ph.fix_ok = 2.0 * bound < std::ldexp(1.0, 51 - g) ? 1 : 0;
  }
}

int alloc_pstate(dpde_handle* h, PState& s) {
  int rc;
  if ((rc = dalloc(h, &s.r, h->n)) || (rc = dalloc(h, &s.eps, h->n))) return rc;
  return DPDE_OK;
}

int allocate(dpde_handle* h) {
  int rc;
  const int64_t n = h->n;
  if ((rc = alloc_pstate(h, h->cur)) || (rc = alloc_pstate(h, h->alt))) return rc;
  if ((rc = dalloc(h, &h->Fx, n)) || (rc = dalloc(h, &h->Fy, n)) || (rc = dalloc(h, &h->Fz, n)) ||
      (rc = dalloc(h, &h->dpi, n)) || (rc = dalloc(h, &h->hv, n)) || (rc = dalloc(h, &h->deps, n)) || (rc = dalloc(h, &h->Ui, n)) ||
      (rc = dalloc(h, &h->Li, n)) ||
      (rc = dalloc(h, &h->idk, n)))
    return rc;
  if ((rc = dalloc(h, &h->key, n)) || (rc = dalloc(h, &h->ticket, n)) ||
      (rc = dalloc(h, &h->bucket, n)))
    return rc;
  if ((rc = dalloc(h, &h->cell_count, h->ncells)) || (rc = dalloc(h, &h->cell_start, h->ncells + 1)))
    return rc;
  h->scan_tiles = (int)((h->ncells + kScanTile - 1) / kScanTile);
  if (h->scan_tiles > 1024 * 8) return fail(DPDE_EINVAL, "too many cells (%lld)", (long long)h->ncells);
  if ((rc = dalloc(h, &h->scan_tmp, h->scan_tiles + 1))) return rc;
  h->nl.stride = n;
  if ((rc = dalloc(h, &h->nl.idx, (size_t)h->phys.cap * n)) || (rc = dalloc(h, &h->nl.count, n)))
    return rc;
  if ((rc = dalloc(h, &h->qid, n)) ||
      (rc = dalloc(h, &h->ctl, 1)) || (rc = dalloc(h, &h->ctl_next, 1)) ||
      (rc = dalloc(h, &h->builds, 1)) ||
      (rc = dalloc(h, &h->skin.idx, (size_t)h->phys.cap * n)) ||
      (rc = dalloc(h, &h->slot, n)) ||
      (rc = dalloc(h, &h->skin.count, n)))
    return rc;
  h->skin.stride = n;
  h->skin.cap = h->phys.cap;
  if (h->hybrid) {
    h->dscan_tiles = (int)((h->ndoms + kScanTile - 1) / kScanTile);
    if (h->dscan_tiles > 1024 * 8) return fail(DPDE_EINVAL, "too many domains");
    h->pscan_tiles = (int)((n + kScanTile - 1) / kScanTile);
    if (h->pscan_tiles > 1024 * 8)
      return fail(DPDE_EINVAL, "Hybrid supports at most %lld particles",
                  (long long)(1024 * 8) * kScanTile);
    // each intra-domain pair is counted once, from its lower identifier: at
    // most half the list entries
    h->ssa.cap = ((int64_t)h->phys.cap * n + 1) / 2;
    if ((rc = dalloc(h, &h->dom, n)) || (rc = dalloc(h, &h->dperm, n)) ||
        (rc = dalloc(h, &h->dbucket, n)) || (rc = dalloc(h, &h->lslot, n)) ||
        (rc = dalloc(h, &h->dcount, h->ndoms + 1)) || (rc = dalloc(h, &h->dstart, h->ndoms + 1)) ||
        (rc = dalloc(h, &h->dscan_tmp, (size_t)h->dscan_tiles + 1)) ||
        (rc = dalloc(h, &h->pcnt, n)) || (rc = dalloc(h, &h->poff, n + 1)) ||
        (rc = dalloc(h, &h->pscan_tmp, (size_t)h->pscan_tiles + 1)) ||
        (rc = dalloc(h, &h->ssa.idx, (size_t)h->ssa.cap)) ||
        (rc = dalloc(h, &h->ssa.gc, (size_t)h->ssa.cap)) ||
        (rc = dalloc(h, &h->always, 1)))
      return rc;
    HIPCHK(hipMemset(h->dcount, 0, (h->ndoms + 1) * sizeof(uint32_t)));
    HIPCHK(hipMemset(h->pcnt, 0, n * sizeof(uint32_t)));
    static const BuildCtl now{0ull, 1u, 0u};
    HIPCHK(hipMemcpy(h->always, &now, sizeof(BuildCtl), hipMemcpyHostToDevice));
  }
  HIPCHK(hipMemset(h->qid, 0, n * sizeof(QIdF)));
  HIPCHK(hipMemset(h->ctl, 0, sizeof(BuildCtl)));
  HIPCHK(hipMemset(h->ctl_next, 0, sizeof(BuildCtl)));
  HIPCHK(hipMemset(h->builds, 0, sizeof(unsigned long long)));
  h->nl.dex = h->nl.dey = h->nl.dez = nullptr;
  if (!h->regen && ((rc = dalloc(h, &h->nl.dex, (size_t)h->phys.cap * n)) ||
                    (rc = dalloc(h, &h->nl.dey, (size_t)h->phys.cap * n)) ||
                    (rc = dalloc(h, &h->nl.dez, (size_t)h->phys.cap * n))))
    return rc;
  if ((rc = dalloc(h, &h->status, 4)) || (rc = dalloc(h, &h->d_step, 1)) ||
      (rc = dalloc(h, &h->d_hist_count, 1)) || (rc = dalloc(h, &h->counter, 1)) ||
      (rc = dalloc(h, &h->stats_ticket, 1)))
    return rc;
  // observable tiles: chunks of kStatTile inside each replica
  std::vector<int64_t> tb;
  std::vector<int32_t> rt;
  for (int r = 0; r < h->nrep; ++r) {
    rt.push_back((int32_t)tb.size());
    for (int64_t b = h->offsets[r]; b < h->offsets[r + 1]; b += kStatTile) tb.push_back(b);
  }
  rt.push_back((int32_t)tb.size());
  h->ntiles = (int)tb.size();
  tb.push_back(n);
  if ((rc = dalloc(h, &h->tile_begin, tb.size())) || (rc = dalloc(h, &h->rep_tile0, rt.size())) ||
      (rc = dalloc(h, &h->partials, (size_t)h->ntiles * kStatVals)) ||
      (rc = dalloc(h, &h->rec, (size_t)h->nrep * kRecLen)) ||
      (rc = dalloc(h, &h->E0, (size_t)h->nrep)))
    return rc;
  HIPCHK(hipMemcpy(h->tile_begin, tb.data(), tb.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(h->rep_tile0, rt.data(), rt.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  {
    // slots of the partial sums the tile sweep 2 adds into, zero between steps
    h->nslots_u = h->batch ? kTailSlotsPerReplica
                           : (int)std::min<int64_t>(kTailSlots, blocks(n, kUniqTile));
    std::vector<int32_t> first(h->nrep + 1);
    for (int r = 0; r <= h->nrep; ++r) first[r] = r * h->nslots_u;
    const size_t total = (size_t)h->nrep * h->nslots_u * kStatVals;
    if ((rc = dalloc(h, &h->partials_u, total)) || (rc = dalloc(h, &h->rep_tile0_u, first.size())))
      return rc;
    HIPCHK(hipMemset(h->partials_u, 0, total * sizeof(Fix)));
    HIPCHK(hipMemcpy(h->rep_tile0_u, first.data(), first.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice));
    h->min_rep_n = n;
    for (int r = 0; r < h->nrep; ++r)
      h->min_rep_n = std::min(h->min_rep_n, h->offsets[r + 1] - h->offsets[r]);
  }
  h->hist_cap = std::max<int64_t>(16, std::min<int64_t>(65536, kHistBytes / (h->nrep * kRecLen * 8)));
  if ((rc = dalloc(h, &h->hist, (size_t)h->hist_cap * h->nrep * kRecLen))) return rc;
  if ((rc = dalloc(h, &h->geo, h->nrep))) return rc;
  HIPCHK(hipMemcpy(h->geo, h->geo_h.data(), h->nrep * sizeof(Geo), hipMemcpyHostToDevice));
  HIPCHK(hipMemset(h->status, 0, 4 * sizeof(uint32_t)));
  HIPCHK(hipMemset(h->cell_count, 0, h->ncells * sizeof(uint32_t)));
  HIPCHK(hipMemset(h->d_hist_count, 0, sizeof(int64_t)));
  HIPCHK(hipMemset(h->stats_ticket, 0, sizeof(uint32_t)));
  return DPDE_OK;
}

int status_to_code(uint32_t st) {
  if (st & ST_NONFINITE) return fail(DPDE_ENONFINITE, "non-finite value in the particle state");
  if (st & ST_NEG_EINT)
    return fail(DPDE_ENEG_EINT, "an internal energy (or temperature) became non-positive");
  if (st & ST_EOS) return fail(DPDE_EEOS, "temperature inversion failed");
  if (st & ST_RANGE)
    return fail(DPDE_ERANGE,
                "a pair term left the range of the fixed-point sums (|dp_ij| or |e_ij| >= 32)");
  if (st & ST_OVERFLOW)
    return fail(DPDE_EOVERFLOW, "a particle has more neighbours than the list capacity");
  return DPDE_OK;
}

// ---- the launch sequence -----------------------------------------------------
// The tile form (the default): pairs inside a 128-particle tile evaluated
// once, every per-particle pair sum in fixed point.  Not for SEM, whose update
// is not written as a sum of stored terms here, nor Hybrid, whose SSA part
// reads full, identifier-ordered lists; and only for the soft potential with
// a < 1024, whose pair force and potential stay inside the range of pass A's
// fixed-point sums (the splined LJ force grows without bound as r -> 0).
bool uniq_form(const dpde_handle* h) {
  return h->pairs_once && h->phys.scheme == DPDE_SCHEME_SER && !h->hybrid &&
         h->phys.potential == DPDE_POT_SOFT && h->phys.a < 1024.0 && h->phys.fix_ok;
}

// The end of the step in the tile sweep 2 (StepTail): without the
// projection, whose observables are taken once, from the state the sweep
// writes; in a batch only when every replica fills a tile (a tile then spans
// at most two replicas).
bool fused_tail(const dpde_handle* h) {
  return uniq_form(h) && !h->phys.project && (!h->batch || h->min_rep_n >= kUniqTile);
}

// What the end of a step's sweep 2 does besides the sweep.
enum TailMode { kTailNone = 0, kTailStats = 1, kTailStatsKick = 2 };

// Kick and drift (unless the previous step's sweep 2 did them: with_kick
// false); on list-build steps (decided on the device) the binning, the
// reorder and the skin lists.  Buffer roles are the same either way.
void enqueue_bin(dpde_handle* h, int kick, bool with_kick = true) {
  const int b = h->aux_block;
  const int64_t n = h->n;
  const double hs2 = h->half_skin2;
  const BuildCtl* ctl = h->ctl;
  if (with_kick)
    launch(h, "kick", h->batch ? k_kick<true> : k_kick<false>, blocks(n, b), b, h->cur,
           (const double*)h->Fx, (const double*)h->Fy, (const double*)h->Fz, n,
           (const Geo*)h->geo, h->phys, kick, (const QIdF*)h->qid, h->ctl, h->status);
  launch(h, "bin_key", h->batch ? k_bin_key<true> : k_bin_key<false>, blocks(n, b), b, h->cur, n,
         (const Geo*)h->geo, h->key, h->ticket, h->idk, h->cell_count, ctl, hs2, h->status);
  launch(h, "scan_tiles", k_scan_tiles, h->scan_tiles, kScanThreads, (const uint32_t*)h->cell_count,
         h->ncells, h->scan_tmp, ctl, hs2);
  launch(h, "scan_apply", k_scan_apply, h->scan_tiles, kScanThreads, h->cell_count, h->ncells,
         (const uint32_t*)h->scan_tmp, h->cell_start, ctl, hs2);
  launch(h, "scatter", k_scatter, blocks(n, b), b, (const uint32_t*)h->key,
         (const uint32_t*)h->ticket, (const uint32_t*)h->cell_start, n, h->bucket, ctl, hs2,
         (const uint32_t*)h->status);
  launch(h, "rank_gather", h->batch ? k_rank_gather<true> : k_rank_gather<false>, blocks(n, b),
         b, h->cur, h->alt, (const uint32_t*)h->bucket, (const uint32_t*)h->cell_start,
         (const uint32_t*)h->key, (const uint32_t*)h->idk, n, (const Geo*)h->geo, h->qid, h->slot,
         ctl, hs2, (const uint32_t*)h->status);
  const int uniq = uniq_form(h) ? 1 : 0;
  const int pb = h->pair_block;
  // the list build reads the reordered records from the spare buffer and
  // returns them to the working one
  launch(h, "build_skin", h->batch ? k_build_skin<true> : k_build_skin<false>,
         blocks(n * kSub, pb), pb, h->alt, h->cur, (const QIdF*)h->qid,
         (const uint32_t*)h->cell_start, n, (const Geo*)h->geo, std::sqrt(h->rs2), h->box_max,
         h->skin, ctl, hs2, uniq, h->status);
  // the tile form adds every pair term in fixed point: its lists need no order
  if (!uniq)
    launch(h, "sort_skin", h->skin.cap > 96 ? k_sort_skin<128> : k_sort_skin<64>,
           blocks(n, 256), 256, n, h->skin, (const uint32_t*)h->slot, ctl, hs2,
           (const uint32_t*)h->status);
}

void enqueue_forces(dpde_handle* h, int mode) {
  const int b = h->pair_block;
  const int64_t n = h->n;
  if (uniq_form(h)) {
    auto go = [&](auto kern) {
      launch(h, "pass_a_forces", kern, blocks(n, kUniqTile), kSub * kUniqTile, h->cur, n,
             (const Geo*)h->geo, h->phys, mode, h->Fx, h->Fy, h->Fz, h->Ui, h->Li, h->skin,
             h->nl, h->status);
    };
    if (h->batch && h->min_rep_n < kWave / kSub) {  // a wave may meet more than two replicas
      if (h->phys.precision == DPDE_FP32) go(k_pass_a_uniq<true, PREC_F32, true>);
      else go(k_pass_a_uniq<true, PREC_F64, true>);
    } else if (h->batch) {
      if (h->phys.precision == DPDE_FP32) go(k_pass_a_uniq<true, PREC_F32>);
      else go(k_pass_a_uniq<true, PREC_F64>);
    } else {
      if (h->phys.precision == DPDE_FP32) go(k_pass_a_uniq<false, PREC_F32>);
      else go(k_pass_a_uniq<false, PREC_F64>);
    }
    return;
  }
  auto go = [&](auto kern) {
    launch(h, "pass_a_forces", kern, blocks(n * kSub, b), b, h->cur, n, (const Geo*)h->geo, h->phys, mode,
           h->Fx, h->Fy, h->Fz, h->Ui, h->Li, h->skin, h->nl, h->status);
  };
  if (h->batch) {
    if (h->phys.precision == DPDE_FP32) go(k_pass_a<true, PREC_F32>);
    else go(k_pass_a<true, PREC_F64>);
  } else {
    if (h->phys.precision == DPDE_FP32) go(k_pass_a<false, PREC_F32>);
    else go(k_pass_a<false, PREC_F64>);
  }
}

bool eos_inline(const dpde_handle* h) {
  return h->phys.eos == DPDE_EOS_LINEAR || h->phys.theta_mode == DPDE_THETA_NEWTON;
}

// Hybrid (Sec. 3.2.2): particles binned by domain and ranked by identifier
// inside it, the intra-domain pairs listed in SSA order with their weights
// and noise, then one lane per domain runs SSA over its pairs.
template <bool B>
void enqueue_hybrid_ssa(dpde_handle* h) {
  const int b = h->aux_block;
  const int64_t n = h->n;
  const BuildCtl* now = h->always;
  launch(h, "dom_key", k_dom_key<B>, blocks(n, b), b, h->cur, n, (const Geo*)h->geo, h->dom,
         h->key, h->ticket, h->idk, h->dcount, (const uint32_t*)h->status);
  // the scan writes dstart[0..ndoms), and dstart[ndoms] = n closes the last domain
  launch(h, "dom_scan_tiles", k_scan_tiles, h->dscan_tiles, kScanThreads,
         (const uint32_t*)h->dcount, h->ndoms, h->dscan_tmp, now, 0.0);
  launch(h, "dom_scan_apply", k_scan_apply, h->dscan_tiles, kScanThreads, h->dcount, h->ndoms,
         (const uint32_t*)h->dscan_tmp, h->dstart, now, 0.0);
  launch(h, "dom_scatter", k_scatter, blocks(n, b), b, (const uint32_t*)h->key,
         (const uint32_t*)h->ticket, (const uint32_t*)h->dstart, n, h->dbucket, now, 0.0,
         (const uint32_t*)h->status);
  launch(h, "dom_rank", k_dom_rank, blocks(n, b), b, (const uint32_t*)h->dbucket,
         (const uint32_t*)h->dstart, (const uint32_t*)h->dom, (const uint32_t*)h->idk, n, h->nl,
         h->dperm, h->lslot, h->pcnt, (const uint32_t*)h->status);
  // poff[k] = first pair of sorted slot k, poff[n] = all pairs
  launch(h, "ssa_scan_tiles", k_scan_tiles, h->pscan_tiles, kScanThreads,
         (const uint32_t*)h->pcnt, n, h->pscan_tmp, now, 0.0);
  launch(h, "ssa_scan_apply", k_scan_apply, h->pscan_tiles, kScanThreads, h->pcnt, n,
         (const uint32_t*)h->pscan_tmp, h->poff, now, 0.0);
  const int pb = h->pair_block;
  launch(h, "ssa_pairs", k_ssa_pairs<B>, blocks(n * kSub, pb), pb, h->cur, h->nl, (const uint32_t*)h->dperm,
         (const uint32_t*)h->lslot, n, (const uint32_t*)h->dom, (const uint32_t*)h->idk,
         (const uint32_t*)h->poff, (const Geo*)h->geo, h->phys, (const uint64_t*)h->d_step, h->ssa,
         h->status);
  auto walk = [&](auto kern) {
    launch(h, "ssa_domains", kern, blocks(h->ndoms, kWave), kWave, h->cur,
           (const uint32_t*)h->dperm, (const uint32_t*)h->dstart, h->ndoms,
           (const uint32_t*)h->poff, h->ssa, h->phys, h->status);
  };
  // LDS slots a wave of domains needs at 1.25 times the mean domain size
  const double need = kWave * 1.25 * (double)n / (double)h->ndoms + 128.0;
  if (need <= 512.0) walk(k_ssa_walk<512>);
  else if (need <= 1024.0) walk(k_ssa_walk<1024>);
  else walk(k_ssa_walk<kSsaPoolMax>);
}

template <bool B, int PR, int MD>
void enqueue_fd_t(dpde_handle* h, TailMode tm) {
  const int b = h->pair_block;
  const int64_t n = h->n;
  const int inl = eos_inline(h) ? 1 : 0;
  const uint64_t* d_step = h->d_step;
  const int store = h->regen ? 0 : 1;
  const uint32_t* dom = h->hybrid ? (const uint32_t*)h->dom : nullptr;
  if (h->hybrid) enqueue_hybrid_ssa<B>(h);
  if (h->phys.scheme == DPDE_SCHEME_SEM) {
    launch(h, "pass_b_sem", k_pass_b<B, PR, 1, MD>, blocks(n * kSubSer, b), b, h->cur, h->nl, n,
           (const Geo*)h->geo, h->phys, d_step, h->dpi, h->hv, h->deps, 0, dom, h->status);
    launch(h, "apply_sem", k_apply_sem, blocks(n, h->aux_block), h->aux_block, h->cur, n, h->phys,
           (const Vec4*)h->dpi, (const double*)h->deps, inl, h->alt.r, h->status);
  } else {
    const bool uq = uniq_form(h);
    if (uq) {
      launch(h, "pass_b_ser", k_pass_b_uniq<B, PR, MD>, blocks(n, kUniqTile), 2 * kUniqTile,
             h->cur, h->nl, n, (const Geo*)h->geo, h->phys, d_step, h->dpi, h->hv, store,
             h->status);
    } else {
      launch(h, "pass_b_ser", k_pass_b<B, PR, 0, MD>, blocks(n * kSubSer, b), b, h->cur, h->nl,
             n, (const Geo*)h->geo, h->phys, d_step, h->dpi, h->hv, h->deps, store, dom,
             h->status);
    }
    // the surrogate's 1/T_i is computed inside sweep 2 (learned-EOS modes)
    const MlpDev m = mlp_dev(h->mlp);
    const int mode = h->mlp.trained ? h->phys.theta_mode : 0;
    auto pass_c = [&](auto kern, unsigned grid, unsigned block) {
      launch(h, "pass_c_ser", kern, grid, block, h->cur, h->nl, n, (const Geo*)h->geo,
             h->phys, d_step, (const Vec4*)h->dpi, (const H3*)h->hv, inl, m, mode, h->alt.r,
             h->status);
    };
    StepTail tail{h->Fx, h->Fy, h->Fz, h->Ui, h->Li, h->qid, h->ctl_next, h->partials_u,
                  h->nslots_u, tm != kTailNone ? 1 : 0, tm == kTailStatsKick ? 1 : 0};
    auto pass_c_uniq = [&](auto kern) {
      launch(h, "pass_c_ser", kern, blocks(n, kUniqTile), 2 * kUniqTile, h->cur, h->nl, n,
             (const Geo*)h->geo, h->phys, d_step, (const Vec4*)h->dpi, (const H3*)h->hv, inl, m,
             mode, h->alt.r, tail, h->status);
    };
    const unsigned go = blocks(n * kSubSer, b), bo = (unsigned)b;
    if (h->regen) {
      if (uq) {
        if (inl) pass_c_uniq(k_pass_c_uniq<B, PR, 1, MD, 0>);
        else pass_c_uniq(k_pass_c_uniq<B, PR, 1, MD, 1>);
      } else {
        if (inl) pass_c(k_pass_c<B, PR, 1, MD, 0>, go, bo);
        else pass_c(k_pass_c<B, PR, 1, MD, 1>, go, bo);
      }
    } else {
      if (uq) {
        if (inl) pass_c_uniq(k_pass_c_uniq<B, PR, 0, MD, 0>);
        else pass_c_uniq(k_pass_c_uniq<B, PR, 0, MD, 1>);
      } else {
        if (inl) pass_c(k_pass_c<B, PR, 0, MD, 0>, go, bo);
        else pass_c(k_pass_c<B, PR, 0, MD, 1>, go, bo);
      }
    }
  }
  // the updated records were written to the spare record array: swap them in
  // (one swap per step, so two steps restore the starting layout, which is
  // what an even-length captured graph relies on)
  std::swap(h->cur.r, h->alt.r);
  if (!inl && h->phys.scheme == DPDE_SCHEME_SEM)
    enqueue_theta_mlp(h->mlp, h->stream, h->cur.eps, &h->cur.r->invT, 8, n, h->phys, h->status);
}

template <bool B, int PR>
void enqueue_fd_m(dpde_handle* h, TailMode tm) {
  if (h->phys.model == DPDE_MODEL_PROJECTED) enqueue_fd_t<B, PR, 1>(h, tm);
  else enqueue_fd_t<B, PR, 0>(h, tm);
}

void enqueue_fd(dpde_handle* h, TailMode tm) {
  if (h->batch) {
    if (h->phys.precision == DPDE_FP32) enqueue_fd_m<true, PREC_F32>(h, tm);
    else enqueue_fd_m<true, PREC_F64>(h, tm);
  } else {
    if (h->phys.precision == DPDE_FP32) enqueue_fd_m<false, PREC_F32>(h, tm);
    else enqueue_fd_m<false, PREC_F64>(h, tm);
  }
}

// With `swept`, the tile sweep 2 has written the partial sums already.
void enqueue_stats_only(dpde_handle* h, int advance, int finish, bool swept = false) {
  if (!swept)
    launch(h, "stats_tiles", k_stats_tiles, h->ntiles, kStatThreads, h->cur,
           (const double*)h->Ui, (const double*)h->Li, (const double*)h->Fx,
           (const double*)h->Fy, (const double*)h->Fz, (const int64_t*)h->tile_begin, h->phys,
           h->partials);
  launch(h, "stats_final", k_stats_final, h->nrep, kStatFinalThreads,
         swept ? h->partials_u : h->partials, swept ? 1 : 0,
         (const int32_t*)(swept ? h->rep_tile0_u : h->rep_tile0), (const Geo*)h->geo, h->d_step,
         advance, h->rec, h->hist, h->hist_cap, h->d_hist_count, h->nrep, finish,
         h->stats_ticket, h->ctl, h->ctl_next, h->builds, h->half_skin2,
         (const uint32_t*)h->status);
}

// Observables of the step; with the projection (Sec. 4.2) the record of the
// unconstrained update gives E, the internal energies are shifted, and the
// record is taken again from the projected state.
void enqueue_stats(dpde_handle* h, int advance, bool swept = false) {
  if (advance && h->phys.project) {
    enqueue_stats_only(h, 0, 0);
    const int inl = eos_inline(h) ? 1 : 0;
    launch(h, "project", h->batch ? k_project<true> : k_project<false>, blocks(h->n, h->aux_block),
           h->aux_block, h->cur, h->n, (const Geo*)h->geo, h->phys, (const double*)h->rec,
           (const double*)h->E0, inl, h->status);
    if (!inl)
      enqueue_theta_mlp(h->mlp, h->stream, h->cur.eps, &h->cur.r->invT, 8, h->n, h->phys,
                        h->status);
  }
  // the last block of the final pass also ends the step
  enqueue_stats_only(h, advance, 1, swept);
}

// One step of a call's sequence.  Where the tile sweep 2 takes the end of the
// step, the kick of every step but the first runs in the previous step's
// sweep 2, and the last step leaves its records unkicked: between calls the
// state is the end of a step, as without the fusion, with the same bits.
void enqueue_step(dpde_handle* h, bool first, bool last) {
  const bool fuse = fused_tail(h);
  enqueue_bin(h, 1, first || !fuse);
  enqueue_forces(h, 1);
  enqueue_fd(h, !fuse ? kTailNone : last ? kTailStats : kTailStatsKick);
  enqueue_stats(h, 1, fuse);
}

void enqueue_steps(dpde_handle* h, int64_t nsteps) {
  for (int64_t s = 0; s < nsteps; ++s) enqueue_step(h, s == 0, s == nsteps - 1);
}

// Bin, forces, temperatures and observables of the current state.
int prepare(dpde_handle* h) {
  HIPCHK(hipMemcpyAsync(h->d_step, &h->step, sizeof(uint64_t), hipMemcpyHostToDevice, h->stream));
  static const BuildCtl forced{0ull, 1u, 0u};
  HIPCHK(hipMemcpyAsync(h->ctl, &forced, sizeof(BuildCtl), hipMemcpyHostToDevice, h->stream));
  enqueue_bin(h, 0);
  enqueue_forces(h, 0);
  if (eos_inline(h)) {
    launch(h, "inv_temperature", k_inv_temperature, blocks(h->n, h->aux_block), h->aux_block,
           h->cur, h->n, h->phys, h->status);
  } else {
    enqueue_theta_mlp(h->mlp, h->stream, h->cur.eps, &h->cur.r->invT, 8, h->n, h->phys, h->status);
  }
  enqueue_stats(h, 0);
  launch(h, "capture_e0", k_capture_e0, blocks(h->nrep, 256), 256, (const double*)h->rec, h->E0,
         h->nrep);
  uint32_t st = 0;
  HIPCHK(hipMemcpyAsync(&st, h->status, sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipGetLastError());
  if (st) {
    int rc = status_to_code(st);
    HIPCHK(hipMemset(h->status, 0, sizeof(uint32_t)));
    return rc;
  }
  return DPDE_OK;
}

int load(dpde_handle* h, const double* q, const double* p, const double* eps) {
  if (!q || !p || !eps) return fail(DPDE_EINVAL, "q, p and eps must be device pointers");
  HIPCHK(hipStreamSynchronize(h->user_stream));
  HIPCHK(hipMemsetAsync(h->status, 0, sizeof(uint32_t), h->stream));
  launch(h, "load_state", k_load_state, blocks(h->n, 256), 256, q, p, eps, (const Geo*)h->geo,
         h->nrep, h->n, h->cur, h->status);
  uint32_t st = 0;
  HIPCHK(hipMemcpyAsync(&st, h->status, sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipGetLastError());
  if (st & ST_NONFINITE) {
    HIPCHK(hipMemset(h->status, 0, sizeof(uint32_t)));
    return fail(DPDE_EINVAL, "non-finite value in the initial state");
  }
  if (st) {
    HIPCHK(hipMemset(h->status, 0, sizeof(uint32_t)));
    return status_to_code(st);
  }
  return DPDE_OK;
}

void release(dpde_handle* h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  for (auto& r : h->prof) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : h->event_pool) (void)hipEventDestroy(e);
  mlp_release(h->mlp);
  for (void* p : h->allocations) (void)hipFree(p);
  if (h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
}

// ---- tuning table -----------------------------------------------------------
struct TuneKey {
  int nclass, rclass, precision;
  bool operator<(const TuneKey& o) const {
    if (nclass != o.nclass) return nclass < o.nclass;
    if (rclass != o.rclass) return rclass < o.rclass;
    return precision < o.precision;
  }
};
struct TuneEntry {
  dpde_shape shape;
  double ms;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune;

int floor_log2(int64_t v) {
  int k = 0;
  while (v > 1) {
    v >>= 1;
    ++k;
  }
  return k;
}

TuneKey tune_key(int64_t n, int32_t nrep, int32_t precision) {
  return TuneKey{floor_log2(n), nrep <= 1 ? 0 : 1 + floor_log2(nrep), precision};
}

bool shape_valid(const dpde_shape& sh) {
  auto ok = [](int b, int mx) { return b >= 64 && b <= mx && (b % 64) == 0; };
  return ok(sh.pair_block, kPairBlockMax) && ok(sh.aux_block, kAuxMaxThreads) &&
         (sh.pairs == DPDE_PAIRS_BOTH_SIDES || sh.pairs == DPDE_PAIRS_ONCE_PER_TILE) &&
         sh.order_block >= 1 && sh.order_block <= kOrderBlockMax;
}

// Shape fields of the handle (host side; the caller uploads the geometry
// and rebuilds the lists where the order or the form changed).
// A captured step graph holds its kernels' arguments (launch shapes, the
// physics block, the surrogate's mode and normalisation): whatever changes
// them drops it, and the next dpde_step_graph captures again.
void drop_graph(dpde_handle* h) {
  if (h->graph_exec) { (void)hipGraphExecDestroy(h->graph_exec); h->graph_exec = nullptr; }
  if (h->graph) { (void)hipGraphDestroy(h->graph); h->graph = nullptr; }
}

void put_shape(dpde_handle* h, const dpde_shape& sh) {
  h->pair_block = sh.pair_block;
  h->aux_block = sh.aux_block;
  h->pairs_once = sh.pairs == DPDE_PAIRS_ONCE_PER_TILE;
  for (Geo& g : h->geo_h) {
    g.oblk = sh.order_block;
    g.oblk_inv = 1.0f / (float)sh.order_block;
  }
  drop_graph(h);
}

dpde_shape get_shape(const dpde_handle* h) {
  dpde_shape sh;
  sh.pair_block = h->pair_block;
  sh.aux_block = h->aux_block;
  sh.pairs = h->pairs_once ? DPDE_PAIRS_ONCE_PER_TILE : DPDE_PAIRS_BOTH_SIDES;
  sh.order_block = h->geo_h[0].oblk;
  return sh;
}

int upload_geo(dpde_handle* h) {
  HIPCHK(hipMemcpyAsync(h->geo, h->geo_h.data(), h->nrep * sizeof(Geo), hipMemcpyHostToDevice,
                        h->stream));
  return DPDE_OK;
}


int create(const dpde_params* params, int nrep, const int64_t* offsets, const double* q,
           const double* p, const double* eps, void* stream, dpde_handle** out) {
  if (!out) return fail(DPDE_EINVAL, "out is NULL");
  *out = nullptr;
  if (nrep < 1) return fail(DPDE_EINVAL, "nrep must be >= 1");
  int rc = check_params(params, true);
  if (rc) return rc;
  dpde_handle* h = new (std::nothrow) dpde_handle();
  if (!h) return fail(DPDE_ENOMEM, "host allocation failed");
  h->nrep = nrep;
  h->batch = nrep > 1;
  h->user_stream = (hipStream_t)stream;
  physics(&params[0], h->phys);
  h->regen = (params[0].flags & DPDE_FLAG_REGENERATE_NOISE) != 0;
  h->half_skin2 = 0.25 * params[0].skin * params[0].skin;
  h->rs2 = (params[0].rc + params[0].skin) * (params[0].rc + params[0].skin);
  h->step = params[0].step0;
  h->offsets.assign(offsets, offsets + nrep + 1);
  if (h->offsets[0] != 0) { release(h); return fail(DPDE_EINVAL, "offsets[0] must be 0"); }
  int64_t cells = 0;
  for (int r = 0; r < nrep; ++r) {
    if ((rc = check_params(&params[r], r == 0))) { release(h); return rc; }
    if (h->offsets[r + 1] - h->offsets[r] != params[r].n) {
      release(h);
      return fail(DPDE_EINVAL, "offsets[%d+1]-offsets[%d] != params[%d].n", r, r, r);
    }
    if (r > 0 && (params[r].mass != params[0].mass || params[r].rc != params[0].rc ||
                  params[r].a != params[0].a || params[r].gamma != params[0].gamma ||
                  params[r].kT_ref != params[0].kT_ref || params[r].dt != params[0].dt ||
                  params[r].eos != params[0].eos || params[r].precision != params[0].precision ||
                  params[r].scheme != params[0].scheme || params[r].step0 != params[0].step0 ||
                  params[r].skin != params[0].skin || params[r].model != params[0].model ||
                  params[r].potential != params[0].potential ||
                  params[r].eps_lj != params[0].eps_lj || params[r].r_lj != params[0].r_lj ||
                  params[r].flags != params[0].flags)) {
      release(h);
      return fail(DPDE_EINVAL, "replica %d: physical parameters differ from replica 0", r);
    }
    Geo g{};
    if ((rc = geometry(&params[r], g))) { release(h); return rc; }
    for (int d = 0; d < 3; ++d) h->box_max = std::max(h->box_max, params[r].box[d]);
    g.cell_base = cells;
    g.first = h->offsets[r];
    g.n = params[r].n;
    cells += (int64_t)g.nc[0] * g.nc[1] * g.nc[2];
    g.dom_base = h->ndoms;
    h->ndoms += (int64_t)g.ndom[0] * g.ndom[1] * g.ndom[2];
    h->geo_h.push_back(g);
  }
  h->n = h->offsets[nrep];
  h->ncells = cells;
  h->hybrid = params[0].scheme == DPDE_SCHEME_HYBRID;
  {  // a shape tuned earlier in this process (or loaded) for this size class
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(tune_key(h->n, nrep, params[0].precision));
    if (it != g_tune.end()) put_shape(h, it->second.shape);
  }
  if (cells >= ((int64_t)1 << 31)) { release(h); return fail(DPDE_EINVAL, "too many cells"); }
  if (h->ndoms >= ((int64_t)1 << 31) / 2) { release(h); return fail(DPDE_EINVAL, "too many domains"); }
  if (hipGetDevice(&h->device) != hipSuccess) { release(h); return fail(DPDE_EHIP, "no HIP device"); }
  if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
    release(h);
    return fail(DPDE_EHIP, "hipStreamCreateWithFlags failed");
  }
  if ((rc = allocate(h))) { release(h); return rc; }
  if ((rc = load(h, q, p, eps))) { release(h); return rc; }
  if ((rc = prepare(h))) { release(h); return rc; }
  *out = h;
  return DPDE_OK;
}

int read_status(dpde_handle* h) {
  uint32_t st = 0;
  HIPCHK(hipMemcpyAsync(&st, h->status, sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipGetLastError());
  if (st) return status_to_code(st);
  return DPDE_OK;
}

// ---- the surrogate gradient without allocation ------------------------------
// One batch's block partials, summed gradient and loss in a fixed device
// array instead of buffers allocated on first use.  In host code `scratch`
// names a host-side stand-in: its device address on each GPU comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr int kNoAllocBlocks = 64;  // block partials of k_mlp_fwd_bwd (its grid is capped at 64)
constexpr size_t kNoAllocGpart = (size_t)kNoAllocBlocks * kNParam * sizeof(float);
constexpr size_t kNoAllocLpart = (size_t)kNoAllocBlocks * sizeof(double);
constexpr size_t kNoAllocGsum = (size_t)kNParam * sizeof(float);
constexpr size_t kNoAllocBytes =
    ((kNoAllocGpart + kNoAllocLpart + kNoAllocGsum + sizeof(float)) + 255) / 256 * 256;
static_assert(kNoAllocGpart % sizeof(double) == 0, "loss partials must stay 8-byte aligned");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (made current by the caller).
int scratch_on(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return fail(DPDE_EINVAL, "device %d out of range", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(DPDE_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", device,
                  hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[device]);
  return DPDE_OK;
}

}  // namespace

extern "C" {

const char* dpde_last_error(void) { return g_last_error.c_str(); }

int dpde_init(const dpde_params* params, const double* q, const double* p, const double* eps,
              void* hip_stream, dpde_handle** out) {
  if (!params) return fail(DPDE_EINVAL, "params is NULL");
  const int64_t offs[2] = {0, params->n};
  return create(params, 1, offs, q, p, eps, hip_stream, out);
}

int dpde_init_batch(const dpde_params* params, int32_t nrep, const int64_t* offsets,
                    const double* q, const double* p, const double* eps, void* hip_stream,
                    dpde_handle** out) {
  if (!params || !offsets) return fail(DPDE_EINVAL, "params and offsets must not be NULL");
  return create(params, nrep, offsets, q, p, eps, hip_stream, out);
}

int dpde_free(dpde_handle* h) {
  release(h);
  return DPDE_OK;
}

void* dpde_stream(dpde_handle* h) { return h ? (void*)h->stream : nullptr; }

int dpde_list_builds(dpde_handle* h, int64_t* builds) {
  if (!h || !builds) return fail(DPDE_EINVAL, "NULL argument");
  unsigned long long b = 0;
  HIPCHK(hipMemcpyAsync(&b, h->builds, sizeof(b), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  *builds = (int64_t)b;
  return DPDE_OK;
}

int dpde_step(dpde_handle* h, int64_t nsteps) {
  if (!h) return fail(DPDE_EINVAL, "handle is NULL");
  if (nsteps < 0) return fail(DPDE_EINVAL, "nsteps < 0");
  enqueue_steps(h, nsteps);
  HIPCHK(hipGetLastError());
  int rc = read_status(h);
  // device step counter is the truth (a failing step stops the counter)
  uint64_t st = 0;
  HIPCHK(hipMemcpy(&st, h->d_step, sizeof(uint64_t), hipMemcpyDeviceToHost));
  h->step = (int64_t)st;
  return rc;
}

int dpde_step_graph(dpde_handle* h, int64_t nsteps, int64_t reps) {
  if (!h) return fail(DPDE_EINVAL, "handle is NULL");
  if (nsteps <= 0 || (nsteps % 2) != 0 || reps < 0)
    return fail(DPDE_EINVAL, "nsteps must be even and > 0, reps >= 0");
  // a graph bakes in the state buffer pointers; eager steps in between can
  // leave the buffers in the other layout, then the graph is captured again
  const bool same_layout = std::memcmp(&h->graph_cur, &h->cur, sizeof(PState)) == 0 &&
                           std::memcmp(&h->graph_alt, &h->alt, sizeof(PState)) == 0;
  if (h->graph_exec == nullptr || h->graph_steps != nsteps || !same_layout) {
    if (h->graph_exec) { (void)hipGraphExecDestroy(h->graph_exec); h->graph_exec = nullptr; }
    if (h->graph) { (void)hipGraphDestroy(h->graph); h->graph = nullptr; }
    const bool prof = h->profiling;
    h->profiling = false;
    HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    // each step swaps the two state buffers; an even count ends where it began,
    // so every replay starts from the same buffers the capture saw
    h->graph_cur = h->cur;
    h->graph_alt = h->alt;
    enqueue_steps(h, nsteps);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->stream, &g);
    h->profiling = prof;
    if (e != hipSuccess) return fail(DPDE_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    h->graph = g;
    HIPCHK(hipGraphInstantiate(&h->graph_exec, g, nullptr, nullptr, 0));
    h->graph_steps = nsteps;
  }
  for (int64_t r = 0; r < reps; ++r) HIPCHK(hipGraphLaunch(h->graph_exec, h->stream));
  int rc = read_status(h);
  uint64_t st = 0;
  HIPCHK(hipMemcpy(&st, h->d_step, sizeof(uint64_t), hipMemcpyDeviceToHost));
  h->step = (int64_t)st;
  return rc;
}

int dpde_energies(dpde_handle* h, double out[DPDE_REC_LEN]) {
  if (!h || !out) return fail(DPDE_EINVAL, "NULL argument");
  HIPCHK(hipMemcpyAsync(out, h->rec, kRecLen * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return DPDE_OK;
}

int dpde_energies_batch(dpde_handle* h, double* out) {
  if (!h || !out) return fail(DPDE_EINVAL, "NULL argument");
  HIPCHK(hipMemcpyAsync(out, h->rec, (size_t)h->nrep * kRecLen * sizeof(double), hipMemcpyDeviceToHost,
                        h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return DPDE_OK;
}

int dpde_history(dpde_handle* h, double* out, int64_t cap, int64_t* count) {
  if (!h || !count) return fail(DPDE_EINVAL, "NULL argument");
  int64_t total = 0;
  HIPCHK(hipMemcpyAsync(&total, h->d_hist_count, sizeof(int64_t), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  const int64_t held = std::min(total, h->hist_cap);
  const int64_t first = total - held;  // oldest record still held
  const int64_t take = std::min(held, cap);
  const size_t rec_doubles = (size_t)h->nrep * kRecLen;
  if (out && take > 0) {
    std::vector<double> buf((size_t)h->hist_cap * rec_doubles);
    HIPCHK(hipMemcpy(buf.data(), h->hist, buf.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < take; ++k) {
      const int64_t slot = (first + k) % h->hist_cap;
      std::memcpy(out + k * rec_doubles, buf.data() + slot * rec_doubles,
                  rec_doubles * sizeof(double));
    }
  }
  *count = take;
  HIPCHK(hipMemset(h->d_hist_count, 0, sizeof(int64_t)));
  return DPDE_OK;
}

int dpde_get_state(dpde_handle* h, double* q, double* p, double* eps, int64_t* step) {
  if (!h) return fail(DPDE_EINVAL, "handle is NULL");
  if (q || p || eps)
    launch(h, "store_state", k_store_state, blocks(h->n, 256), 256, h->cur, (const Geo*)h->geo,
           h->n, q, p, eps);
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipGetLastError());
  if (step) *step = h->step;
  return DPDE_OK;
}

int dpde_set_state(dpde_handle* h, const double* q, const double* p, const double* eps,
                   int64_t step) {
  if (!h) return fail(DPDE_EINVAL, "handle is NULL");
  int rc = load(h, q, p, eps);
  if (rc) return rc;
  h->step = step;
  return prepare(h);
}

int dpde_forces(dpde_handle* h, double* F, double* U) {
  if (!h || !F) return fail(DPDE_EINVAL, "NULL argument");
  launch(h, "store_forces", k_store_vec3, blocks(h->n, 256), 256, h->cur, (const Geo*)h->geo,
         h->n, (const double*)h->Fx, (const double*)h->Fy, (const double*)h->Fz, F);
  double rec[kRecLen];
  HIPCHK(hipMemcpyAsync(rec, h->rec, sizeof(rec), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipGetLastError());
  if (U) *U = rec[0];
  return DPDE_OK;
}

int dpde_tuning_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  return DPDE_OK;
}

int dpde_tuning_lookup(int64_t n, int32_t nrep, int32_t precision, dpde_shape* shape,
                       double* ms_per_step, int32_t* found) {
  if (!found) return fail(DPDE_EINVAL, "found is NULL");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(tune_key(n, nrep, precision));
  *found = it != g_tune.end();
  if (*found) {
    if (shape) *shape = it->second.shape;
    if (ms_per_step) *ms_per_step = it->second.ms;
  }
  return DPDE_OK;
}

int dpde_tuning_save(const char* path) {
  if (!path) return fail(DPDE_EINVAL, "path is NULL");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(DPDE_EIO, "cannot write %s", path);
  std::fprintf(f, "# nclass rclass precision pair_block aux_block pairs order_block ms_per_step\n");
  for (const auto& kv : g_tune)
    std::fprintf(f, "%d %d %d %d %d %d %d %.6f\n", kv.first.nclass, kv.first.rclass,
                 kv.first.precision, kv.second.shape.pair_block, kv.second.shape.aux_block,
                 kv.second.shape.pairs, kv.second.shape.order_block, kv.second.ms);
  const bool bad = std::ferror(f) != 0;
  if (std::fclose(f) != 0 || bad) return fail(DPDE_EIO, "cannot write %s", path);
  return DPDE_OK;
}

int dpde_tuning_load(const char* path) {
  if (!path) return fail(DPDE_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(DPDE_EIO, "cannot read %s", path);
  std::map<TuneKey, TuneEntry> got;
  char line[512];
  int lineno = 0;
  while (std::fgets(line, sizeof line, f)) {
    ++lineno;
    const char* c = line;
    while (*c == ' ' || *c == '\t') ++c;
    if (*c == '#' || *c == '\n' || *c == '\0') continue;
    TuneKey k{};
    TuneEntry e{};
    char tail = 0;
    const int m = std::sscanf(c, "%d %d %d %d %d %d %d %lf %c", &k.nclass, &k.rclass,
                              &k.precision, &e.shape.pair_block, &e.shape.aux_block,
                              &e.shape.pairs, &e.shape.order_block, &e.ms, &tail);
    if (m != 8) {
      std::fclose(f);
      return fail(DPDE_EIO, "%s:%d: expected 8 fields", path, lineno);
    }
    if (!shape_valid(e.shape) || k.nclass < 0 || k.nclass > 62 || k.rclass < 0 ||
        (k.precision != DPDE_FP64 && k.precision != DPDE_FP32)) {
      std::fclose(f);
      return fail(DPDE_EINVAL, "%s:%d: entry out of range", path, lineno);
    }
    got[k] = e;
  }
  std::fclose(f);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& kv : got) g_tune[kv.first] = kv.second;
  return DPDE_OK;
}

int dpde_set_tuning(dpde_handle* h, int32_t pair_block, int32_t aux_block) {
  if (!h) return fail(DPDE_EINVAL, "handle is NULL");
  dpde_shape sh = get_shape(h);
  sh.pair_block = pair_block;
  sh.aux_block = aux_block;
  if (!shape_valid(sh))
    return fail(DPDE_EINVAL, "block sizes must be multiples of 64 within the kernel limits");
  put_shape(h, sh);
  return DPDE_OK;
}

int dpde_get_shape(dpde_handle* h, dpde_shape* out) {
  if (!h || !out) return fail(DPDE_EINVAL, "NULL argument");
  *out = get_shape(h);
  return DPDE_OK;
}

int dpde_set_shape(dpde_handle* h, const dpde_shape* shape) {
  if (!h || !shape) return fail(DPDE_EINVAL, "NULL argument");
  if (shape->pairs != DPDE_PAIRS_BOTH_SIDES && shape->pairs != DPDE_PAIRS_ONCE_PER_TILE)
    return fail(DPDE_EINVAL, "unknown pair form %d", shape->pairs);
  if (shape->order_block < 1 || shape->order_block > kOrderBlockMax)
    return fail(DPDE_EINVAL, "order_block must be in [1, %d], got %d", kOrderBlockMax,
                shape->order_block);
  if (!shape_valid(*shape))
    return fail(DPDE_EINVAL, "block sizes must be multiples of 64 within the kernel limits");
  const dpde_shape cur = get_shape(h);
  put_shape(h, *shape);
  // the order and the lists follow the shape: rebuild them and the forces
  // from the current positions (no kick)
  if (cur.pairs != shape->pairs || cur.order_block != shape->order_block) {
    static const BuildCtl forced{0ull, 1u, 0u, 0ull};
    static const BuildCtl cleared{0ull, 0u, 0u, 0ull};
    int rc = upload_geo(h);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(h->ctl, &forced, sizeof(BuildCtl), hipMemcpyHostToDevice, h->stream));
    enqueue_bin(h, 0);
    enqueue_forces(h, 0);
    HIPCHK(hipMemcpyAsync(h->ctl, &cleared, sizeof(BuildCtl), hipMemcpyHostToDevice, h->stream));
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  return read_status(h);
}

int dpde_autotune(dpde_handle* h, int32_t steps, int32_t* pair_block, int32_t* aux_block,
                  double* ms_per_step) {
  if (!h) return fail(DPDE_EINVAL, "handle is NULL");
  if (steps < 1) return fail(DPDE_EINVAL, "steps must be >= 1");
  // snapshot: state in identifier order, step, list-build count, history
  const size_t n = (size_t)h->n;
  const size_t hist_bytes = (size_t)h->hist_cap * h->nrep * kRecLen * sizeof(double);
  double *q = nullptr, *p = nullptr, *e = nullptr, *hist = nullptr;
  auto cleanup = [&]() {
    if (q) (void)hipFree(q);
    if (p) (void)hipFree(p);
    if (e) (void)hipFree(e);
    if (hist) (void)hipFree(hist);
  };
  if (hipMalloc((void**)&q, 3 * n * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&p, 3 * n * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&e, n * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&hist, hist_bytes) != hipSuccess) {
    cleanup();
    return fail(DPDE_ENOMEM, "autotune snapshot allocation failed");
  }
  int rc = dpde_get_state(h, q, p, e, nullptr);
  const int64_t step0 = h->step;
  int64_t hist_count = 0;
  unsigned long long builds = 0;
  if (!rc) {
    if (hipMemcpyAsync(&hist_count, h->d_hist_count, sizeof(int64_t), hipMemcpyDeviceToHost,
                       h->stream) != hipSuccess ||
        hipMemcpyAsync(&builds, h->builds, sizeof(builds), hipMemcpyDeviceToHost, h->stream) !=
            hipSuccess ||
        hipMemcpyAsync(hist, h->hist, hist_bytes, hipMemcpyDeviceToDevice, h->stream) !=
            hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
      rc = fail(DPDE_EHIP, "autotune snapshot copy failed");
  }
  auto restore = [&]() -> int {
    int r = dpde_set_state(h, q, p, e, step0);
    if (r) return r;
    if (hipMemcpyAsync(h->d_hist_count, &hist_count, sizeof(int64_t), hipMemcpyHostToDevice,
                       h->stream) != hipSuccess ||
        hipMemcpyAsync(h->builds, &builds, sizeof(builds), hipMemcpyHostToDevice, h->stream) !=
            hipSuccess ||
        hipMemcpyAsync(h->hist, hist, hist_bytes, hipMemcpyDeviceToDevice, h->stream) !=
            hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
      return fail(DPDE_EHIP, "autotune restore copy failed");
    return DPDE_OK;
  };
  // candidates: the pair form where the tile form applies, the cell order,
  // the lane-group and per-particle blocks
  const dpde_shape sh0 = get_shape(h);
  std::vector<dpde_shape> cands;
  const bool two_forms = [&] {
    const bool keep = h->pairs_once;
    h->pairs_once = true;
    const bool u = uniq_form(h);
    h->pairs_once = keep;
    return u;
  }();
  for (int form : {DPDE_PAIRS_ONCE_PER_TILE, DPDE_PAIRS_BOTH_SIDES}) {
    if (!two_forms && form != sh0.pairs) continue;
    for (int ob = 1; ob <= 4; ++ob)
      for (int pb : {64, 128, 256})
        for (int ab : {128, 256, 512}) cands.push_back(dpde_shape{pb, ab, form, ob});
  }
  dpde_shape best_sh = sh0;
  double best = 1e300;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (!rc && (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess))
    rc = fail(DPDE_EHIP, "autotune event creation failed");
  for (const dpde_shape& sh : cands) {
    if (rc) break;
    // the shape, then the snapshot state binned and listed under it
    put_shape(h, sh);
    if ((rc = upload_geo(h)) || (rc = restore())) break;
    enqueue_steps(h, 1);  // warm-up (first launch of this shape)
    (void)hipEventRecord(t0, h->stream);
    enqueue_steps(h, steps);
    (void)hipEventRecord(t1, h->stream);
    if (hipEventSynchronize(t1) != hipSuccess) {
      rc = fail(DPDE_EHIP, "autotune timing failed");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, t0, t1);
    rc = read_status(h);
    if (rc) break;
    if (ms / steps < best) {
      best = ms / steps;
      best_sh = sh;
    }
  }
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  // the winner (or, after a failure, the original shape) on the snapshot
  put_shape(h, rc ? sh0 : best_sh);
  int rc2 = upload_geo(h);
  if (!rc2) rc2 = restore();
  cleanup();
  if (rc) return rc;
  if (rc2) return rc2;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[tune_key(h->n, h->nrep, h->phys.precision)] = TuneEntry{best_sh, best};
  }
  if (pair_block) *pair_block = best_sh.pair_block;
  if (aux_block) *aux_block = best_sh.aux_block;
  if (ms_per_step) *ms_per_step = best;
  return DPDE_OK;
}

int dpde_profile_enable(dpde_handle* h, int32_t enable) {
  if (!h) return fail(DPDE_EINVAL, "handle is NULL");
  h->profiling = enable != 0;
  return DPDE_OK;
}

int dpde_profile_read(dpde_handle* h, char* names, double* total_ms, int64_t* launches,
                      int32_t nmax) {
  if (!h) return fail(DPDE_EINVAL, "handle is NULL");
  HIPCHK(hipStreamSynchronize(h->stream));
  std::vector<std::string> order;
  std::map<std::string, std::pair<double, int64_t>> acc;
  for (auto& r : h->prof) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    auto it = acc.find(r.name);
    if (it == acc.end()) {
      order.push_back(r.name);
      acc[r.name] = {ms, 1};
    } else {
      it->second.first += ms;
      it->second.second += 1;
    }
    h->event_pool.push_back(r.a);
    h->event_pool.push_back(r.b);
  }
  h->prof.clear();
  int k = 0;
  for (auto& nm : order) {
    if (k >= nmax) break;
    if (names) {
      std::memset(names + 32 * k, 0, 32);
      std::strncpy(names + 32 * k, nm.c_str(), 31);
    }
    if (total_ms) total_ms[k] = acc[nm].first;
    if (launches) launches[k] = acc[nm].second;
    ++k;
  }
  return k;
}

int dpde_theta(dpde_handle* h, const double* eps, double* theta, int32_t* iters, int64_t n,
               int32_t mode) {
  if (!h || !eps || !theta) return fail(DPDE_EINVAL, "NULL argument");
  if (n < 0 || mode < 0 || mode > 2) return fail(DPDE_EINVAL, "bad n or mode");
  if (mode != DPDE_THETA_NEWTON && !h->mlp.trained)
    return fail(DPDE_EINVAL, "the surrogate has not been trained or set");
  launch_theta(h->mlp, h->stream, eps, theta, iters, n, h->phys, mode);
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipGetLastError());
  return DPDE_OK;
}

int dpde_eos_energy(dpde_handle* h, const double* theta, double* eps, int64_t n) {
  if (!h || !theta || !eps) return fail(DPDE_EINVAL, "NULL argument");
  launch(h, "eos_energy", k_eos_energy, blocks(n, 256), 256, theta, eps, n, h->phys);
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipGetLastError());
  return DPDE_OK;
}

int dpde_mlp_train(dpde_handle* h, const dpde_mlp_cfg* cfg, float* loss_curve) {
  if (!h || !cfg) return fail(DPDE_EINVAL, "NULL argument");
  if (h->phys.eos != DPDE_EOS_EINSTEIN)
    return fail(DPDE_EINVAL, "the surrogate is for the nonlinear (Einstein) EOS");
  std::string err;
  int rc = mlp_train(h->mlp, h->stream, h->phys, *cfg, loss_curve, err);
  if (rc) return fail(rc, "%s", err.c_str());
  mlp_attach(h->mlp, h->phys);
  drop_graph(h);
  return DPDE_OK;
}

int dpde_mlp_get(dpde_handle* h, float* weights, double* norm4) {
  if (!h) return fail(DPDE_EINVAL, "NULL argument");
  std::string err;
  int rc = mlp_get(h->mlp, weights, norm4, err);
  return rc ? fail(rc, "%s", err.c_str()) : DPDE_OK;
}

int dpde_mlp_set(dpde_handle* h, const float* weights, const double* norm4) {
  if (!h || !weights || !norm4) return fail(DPDE_EINVAL, "NULL argument");
  std::string err;
  int rc = mlp_set(h->mlp, h->phys, weights, norm4, err);
  if (rc) return fail(rc, "%s", err.c_str());
  mlp_attach(h->mlp, h->phys);
  drop_graph(h);
  return DPDE_OK;
}

int dpde_mlp_grad(dpde_handle* h, const float* x, const float* t, int64_t n, float* loss,
                  float* grad) {
  if (!h || !x || !t || !loss || !grad) return fail(DPDE_EINVAL, "NULL argument");
  std::string err;
  int rc = mlp_grad(h->mlp, h->stream, x, t, n, loss, grad, err);
  return rc ? fail(rc, "%s", err.c_str()) : DPDE_OK;
}

int dpde_mlp_grad_noalloc(dpde_handle* h, const float* x, const float* t, int64_t n, float* loss,
                          float* grad) {
  if (!h || !x || !t || !loss || !grad) return fail(DPDE_EINVAL, "NULL argument");
  if (n <= 0 || n > DPDE_MLP_GRAD_NOALLOC_MAX_N)
    return fail(DPDE_EINVAL, "n = %lld outside [1, %lld] for dpde_mlp_grad_noalloc", (long long)n,
                (long long)DPDE_MLP_GRAD_NOALLOC_MAX_N);
  if (!h->mlp.w) return fail(DPDE_EINVAL, "the surrogate has no weights");
  HIPCHK(hipSetDevice(h->device));
  unsigned char* base = nullptr;
  int rc = scratch_on(h->device, &base);
  if (rc) return rc;
  float* gpart = reinterpret_cast<float*>(base);
  double* lpart = reinterpret_cast<double*>(base + kNoAllocGpart);
  float* gsum = reinterpret_cast<float*>(base + kNoAllocGpart + kNoAllocLpart);
  float* lsum = reinterpret_cast<float*>(base + kNoAllocGpart + kNoAllocLpart + kNoAllocGsum);
  // the launch shape of dpde_mlp_grad, so both give the same bits; every
  // scratch word read below is written first by this call
  const int gb = (int)std::min<int64_t>(kNoAllocBlocks, (n + kTrainThreads - 1) / kTrainThreads);
  hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3(gb), dim3(kTrainThreads), 0, h->stream,
                     (const float*)h->mlp.w, x, t, n, (int64_t)0, n, 1.0f / (float)n, gpart, lpart);
  hipLaunchKernelGGL(k_mlp_reduce_adam, dim3(1), dim3(1024), 0, h->stream, (const float*)gpart,
                     (const double*)lpart, gb, n, h->mlp.w, h->mlp.adam_m, h->mlp.adam_v,
                     h->mlp.wb, 0.0f, 1.0f, 1.0f, 0, gsum, lsum);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(grad, gsum, kNParam * sizeof(float), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(loss, lsum, sizeof(float), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return DPDE_OK;
}

int dpde_mlp_eval(dpde_handle* h, const float* x, float* y, int64_t n) {
  if (!h || !x || !y) return fail(DPDE_EINVAL, "NULL argument");
  std::string err;
  int rc = mlp_eval(h->mlp, h->stream, x, y, n, err);
  return rc ? fail(rc, "%s", err.c_str()) : DPDE_OK;
}

int dpde_debug_cells(dpde_handle* h, int32_t* cell_of_id) {
  if (!h || !cell_of_id) return fail(DPDE_EINVAL, "NULL argument");
  launch(h, "debug_cells", k_debug_cells, blocks(h->n, 256), 256, h->cur, h->n,
         (const Geo*)h->geo, cell_of_id);
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipGetLastError());
  return DPDE_OK;
}

int dpde_debug_order(dpde_handle* h, int32_t* row_of_slot) {
  if (!h || !row_of_slot) return fail(DPDE_EINVAL, "NULL argument");
  launch(h, "debug_order", k_debug_order, blocks(h->n, 256), 256, h->cur, h->n,
         (const Geo*)h->geo, row_of_slot);
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipGetLastError());
  return DPDE_OK;
}

int dpde_debug_inv_temperature(dpde_handle* h, double* inv_t) {
  if (!h || !inv_t) return fail(DPDE_EINVAL, "NULL argument");
  launch(h, "debug_inv_temperature", k_store_inv_temperature, blocks(h->n, 256), 256, h->cur,
         (const Geo*)h->geo, h->n, inv_t);
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipGetLastError());
  return DPDE_OK;
}

int dpde_debug_list_lengths(dpde_handle* h, int32_t* lengths) {
  if (!h || !lengths) return fail(DPDE_EINVAL, "NULL argument");
  launch(h, "debug_list_lengths", k_store_list_length, blocks(h->n, 256), 256, h->cur,
         (const Geo*)h->geo, h->n, (const uint32_t*)h->nl.count, lengths);
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipGetLastError());
  return DPDE_OK;
}

int dpde_debug_pairs(dpde_handle* h, int32_t* lohi, int64_t cap, int64_t* npairs) {
  if (!h || !npairs || (cap > 0 && !lohi)) return fail(DPDE_EINVAL, "NULL argument");
  HIPCHK(hipMemsetAsync(h->counter, 0, sizeof(unsigned long long), h->stream));
  launch(h, "debug_pairs", k_debug_pairs, blocks(h->n, 256), 256, h->cur, h->nl, h->n,
         (const Geo*)h->geo, uniq_form(h) ? 1 : 0, lohi, cap, h->counter);
  unsigned long long c = 0;
  HIPCHK(hipMemcpyAsync(&c, h->counter, sizeof(c), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipGetLastError());
  *npairs = (int64_t)c;
  return DPDE_OK;
}

int dpde_debug_rng(uint64_t seed, uint32_t replica, int64_t step, const uint32_t* lo,
                   const uint32_t* hi, int64_t n, uint32_t* raw, double* g, float* g32) {
  if (!lo || !hi || n < 0) return fail(DPDE_EINVAL, "bad argument");
  if (n == 0) return DPDE_OK;
  hipLaunchKernelGGL(k_debug_rng, dim3(blocks(n, 256)), dim3(256), 0, nullptr, (uint32_t)seed,
                     (uint32_t)(seed >> 32) ^ replica, (uint64_t)step, lo, hi, n, raw, g, g32);
  HIPCHK(hipGetLastError());
  HIPCHK(hipDeviceSynchronize());
  return DPDE_OK;
}

}  // extern "C"
