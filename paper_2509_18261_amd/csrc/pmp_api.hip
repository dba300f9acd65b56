// Host side of libpmp: context, geometry checks, ghost-fold plan, HIP graph
// capture, tuning and the C-ABI entry points declared in include/pmp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pmp_internal.h"

using namespace pmp;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char msg[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(msg, sizeof msg, fmt, ap);
  va_end(ap);
  g_last_error = msg;
  return code;
}

#define PMP_HIP(call)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(PMP_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));             \
  } while (0)

template <class T> hipError_t dev_alloc(T** p, size_t count) {
  return hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T));
}

struct HostBox {
  int lo[3], n[3];
};

long long shell_count(const int n[3], int g) {
  const int glz = std::min(g, n[2]), hsz = std::max(glz, n[2] - g), nbz = glz + (n[2] - hsz);
  const int gly = std::min(g, n[1]), hsy = std::max(gly, n[1] - g), nby = gly + (n[1] - hsy);
  const int glx = std::min(g, n[0]), hsx = std::max(glx, n[0] - g), nbx = glx + (n[0] - hsx);
  return (long long)nbz * n[0] * n[1] + (long long)(hsz - glz) * nby * n[0] +
         (long long)(hsz - glz) * (hsy - gly) * nbx;
}

// Uniform coarse grid over the domain for box lookups by rectangle.
struct BoxIndex {
  int cell[3], dims[3];
  std::vector<std::vector<int>> bins;
  std::vector<int> stamp;
  int epoch = 0;

  void build(const std::vector<HostBox>& boxes, const int domain[3]) {
    for (int a = 0; a < 3; ++a) {
      int m = 1;
      for (const auto& b : boxes) m = std::max(m, b.n[a]);
      cell[a] = m;
      dims[a] = (domain[a] + m - 1) / m;
    }
    bins.assign((size_t)dims[0] * dims[1] * dims[2], {});
    for (int i = 0; i < (int)boxes.size(); ++i) {
      int c0[3], c1[3];
      for (int a = 0; a < 3; ++a) {
        c0[a] = boxes[i].lo[a] / cell[a];
        c1[a] = (boxes[i].lo[a] + boxes[i].n[a] - 1) / cell[a];
      }
      for (int z = c0[2]; z <= c1[2]; ++z)
        for (int y = c0[1]; y <= c1[1]; ++y)
          for (int x = c0[0]; x <= c1[0]; ++x)
            bins[((size_t)z * dims[1] + y) * dims[0] + x].push_back(i);
    }
    stamp.assign(boxes.size(), -1);
  }

  // Boxes whose owned region intersects [lo, hi) (already clipped to the domain).
  template <class F> void query(const int lo[3], const int hi[3], F&& f) {
    ++epoch;
    int c0[3], c1[3];
    for (int a = 0; a < 3; ++a) {
      c0[a] = lo[a] / cell[a];
      c1[a] = (hi[a] - 1) / cell[a];
    }
    for (int z = c0[2]; z <= c1[2]; ++z)
      for (int y = c0[1]; y <= c1[1]; ++y)
        for (int x = c0[0]; x <= c1[0]; ++x)
          for (int b : bins[((size_t)z * dims[1] + y) * dims[0] + x]) {
            if (stamp[b] == epoch) continue;
            stamp[b] = epoch;
            f(b);
          }
  }
};

struct SegKey {
  int lo[3], s[3];
  DevSeg seg;
};

}  // namespace

struct pmp_ctx {
  int device = 0;
  int nbox = 0, ghost = 0, domain[3] = {0, 0, 0};
  double dx = 1.0, V = 1.0;
  int acc = 0, state = 0, nfield = 5;
  std::vector<HostBox> hboxes;
  std::vector<DevBox> dboxes;
  long long state_elems = 0, buffer_elems = 0, owned_cells = 0, shell_cells = 0;
  int nseg = 0;
  // device allocations
  DevBox* d_boxes = nullptr;
  long long* d_owned_prefix = nullptr;
  long long* d_shell_prefix = nullptr;
  int* d_seg_off = nullptr;
  DevSeg* d_segs = nullptr;
  DevStatus* d_status = nullptr;
  double* d_sink_scratch = nullptr;
  long long sink_cap = 0;
  int num_cu = 256;
  pmp_tuning tune{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  // phase profiler: events[phase][2 * launch + {0: start, 1: stop}]
  bool prof_on = false;
  int prof_max = 0;
  int prof_count[PMP_NPHASE] = {0};
  std::vector<hipEvent_t> prof_events[PMP_NPHASE];

  Mesh mesh() const {
    Mesh M;
    M.boxes = d_boxes;
    M.nbox = nbox;
    M.ghost = ghost;
    for (int a = 0; a < 3; ++a) M.domain[a] = domain[a];
    M.V = V;
    M.nfield = nfield;
    M.acc = acc;
    M.state = state;
    M.buffer_elems = buffer_elems;
    M.owned_cells = owned_cells;
    M.owned_prefix = d_owned_prefix;
    M.shell_prefix = d_shell_prefix;
    M.seg_off = d_seg_off;
    M.segs = d_segs;
    M.shell_cells = shell_cells;
    M.status = d_status;
    M.num_cu = num_cu;
    return M;
  }
  size_t acc_bytes() const { return acc == PMP_ACC_F32 ? 4 : 8; }
};

namespace {

void prof_free(pmp_ctx* c) {
  for (int p = 0; p < PMP_NPHASE; ++p) {
    for (hipEvent_t e : c->prof_events[p]) (void)hipEventDestroy(e);
    c->prof_events[p].clear();
    c->prof_count[p] = 0;
  }
  c->prof_on = false;
  c->prof_max = 0;
}

bool capturing(hipStream_t s);

// Bracket one kernel launch with events when profiling (never under capture).
struct PhaseTimer {
  pmp_ctx* c;
  int phase;
  hipStream_t s;
  bool on;
  PhaseTimer(pmp_ctx* c_, int p, hipStream_t s_) : c(c_), phase(p), s(s_) {
    on = c->prof_on && c->prof_count[p] < c->prof_max && !capturing(s);
    if (on) (void)hipEventRecord(c->prof_events[p][2 * c->prof_count[p]], s);
  }
  ~PhaseTimer() {
    if (on) {
      (void)hipEventRecord(c->prof_events[phase][2 * c->prof_count[phase] + 1], s);
      ++c->prof_count[phase];
    }
  }
};

void release(pmp_ctx* c) {
  prof_free(c);
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  (void)hipFree(c->d_boxes);
  (void)hipFree(c->d_owned_prefix);
  (void)hipFree(c->d_shell_prefix);
  (void)hipFree(c->d_seg_off);
  (void)hipFree(c->d_segs);
  (void)hipFree(c->d_status);
  (void)hipFree(c->d_sink_scratch);
}

// Fold plan (Sec. 2.2 Step 2): for every destination box b and every source
// box b' with periodic shift s, the owned cells of b whose image under +s*D
// lies in the padded box of b' receive those ghost cells.  Per destination
// the segments are ordered by (lo_z', lo_y', lo_x', s_z, s_y, s_x), which is
// the order in which each owned cell adds its contributions (App. A.2).
int build_fold_plan(pmp_ctx* c, std::vector<int>& seg_off, std::vector<DevSeg>& segs) {
  const int g = c->ghost;
  BoxIndex idx;
  idx.build(c->hboxes, c->domain);
  std::vector<std::vector<SegKey>> per(c->nbox);
  int S[3];
  for (int a = 0; a < 3; ++a) S[a] = (g + c->domain[a] - 1) / c->domain[a];
  for (int bs = 0; bs < c->nbox; ++bs) {
    const HostBox& src = c->hboxes[bs];
    for (int sz = -S[2]; sz <= S[2]; ++sz)
      for (int sy = -S[1]; sy <= S[1]; ++sy)
        for (int sx = -S[0]; sx <= S[0]; ++sx) {
          const int s[3] = {sx, sy, sz};
          int lo[3], hi[3];
          bool empty = false;
          for (int a = 0; a < 3; ++a) {
            // padded source box shifted back by s*D, clipped to the domain
            lo[a] = std::max(0, src.lo[a] - g - s[a] * c->domain[a]);
            hi[a] = std::min(c->domain[a], src.lo[a] + src.n[a] + g - s[a] * c->domain[a]);
            if (lo[a] >= hi[a]) empty = true;
          }
          if (empty) continue;
          const bool zero_shift = (sx == 0 && sy == 0 && sz == 0);
          idx.query(lo, hi, [&](int bd) {
            if (bd == bs && zero_shift) return;
            const HostBox& dst = c->hboxes[bd];
            SegKey k;
            for (int a = 0; a < 3; ++a) {
              const int l = std::max(lo[a], dst.lo[a]);
              const int h = std::min(hi[a], dst.lo[a] + dst.n[a]);
              if (l >= h) return;
              k.seg.lo[a] = l - dst.lo[a];
              k.seg.hi[a] = h - dst.lo[a];
              k.seg.off[a] = dst.lo[a] + s[a] * c->domain[a] - src.lo[a] + g;
              k.lo[a] = src.lo[a];
              k.s[a] = s[a];
            }
            k.seg.src = bs;
            per[bd].push_back(k);
          });
        }
  }
  seg_off.assign(c->nbox + 1, 0);
  segs.clear();
  for (int b = 0; b < c->nbox; ++b) {
    auto& v = per[b];
    std::sort(v.begin(), v.end(), [](const SegKey& x, const SegKey& y) {
      const int kx[6] = {x.lo[2], x.lo[1], x.lo[0], x.s[2], x.s[1], x.s[0]};
      const int ky[6] = {y.lo[2], y.lo[1], y.lo[0], y.s[2], y.s[1], y.s[0]};
      return std::lexicographical_compare(kx, kx + 6, ky, ky + 6);
    });
    for (auto& k : v) segs.push_back(k.seg);
    seg_off[b + 1] = (int)segs.size();
  }
  return PMP_OK;
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
  return st == hipStreamCaptureStatusActive;
}

int ensure_sink_scratch(pmp_ctx* c, long long n, hipStream_t s) {
  if (n <= c->sink_cap) return PMP_OK;
  if (capturing(s))
    return fail(PMP_EINVAL, "sink scratch must be sized before graph capture");
  (void)hipFree(c->d_sink_scratch);
  c->d_sink_scratch = nullptr;
  c->sink_cap = 0;
  PMP_HIP(dev_alloc(&c->d_sink_scratch, (size_t)(2 * n)));
  c->sink_cap = n;
  return PMP_OK;
}

Limits to_limits(const pmp_limits* L) {
  Limits l;
  l.rho_floor = L->rho_floor;
  l.rho_tr = L->rho_tr;
  l.cap = L->cap;
  l.eint_mode = L->eint_mode;
  return l;
}

int check_limits(const pmp_limits* L) {
  if (!L) return fail(PMP_EINVAL, "limits is NULL");
  if (!(L->cap >= 0.0) || !(L->rho_floor >= 0.0) || std::isnan(L->rho_tr))
    return fail(PMP_EINVAL, "bad limits (cap %g, rho_floor %g, rho_tr %g)", L->cap,
                L->rho_floor, L->rho_tr);
  if (L->eint_mode != 0 && L->eint_mode != 1)
    return fail(PMP_EINVAL, "eint_mode must be 0 or 1");
  return PMP_OK;
}

int check_sinks(const pmp_ctx* c, const pmp_sinks* k) {
  if (!k->x || !k->y || !k->z || !k->a || !k->box_off)
    return fail(PMP_EINVAL, "sink arrays must be non-NULL");
  if (!c->nfield || c->nfield != 6)
    return fail(PMP_EINVAL, "sinks need a layout created with with_sinks = 1");
  if (c->nbox != 1)
    return fail(PMP_EUNSUPPORTED, "sinks are supported on single-box layouts only");
  for (int a = 0; a < 3; ++a)
    if (c->hboxes[0].lo[a] != 0 || c->hboxes[0].n[a] != c->domain[a])
      return fail(PMP_EUNSUPPORTED, "sinks need the single box to cover the domain");
  if (!(k->r_k >= 0.0) || !(k->r_gauss > 0.0))
    return fail(PMP_EINVAL, "sink radii must satisfy r_k >= 0, r_gauss > 0");
  if (std::floor(k->r_k + 0.5) > c->ghost)
    return fail(PMP_ERANGE, "sink kernel reach floor(r_k + 1/2) = %g exceeds ghost width %d",
                std::floor(k->r_k + 0.5), c->ghost);
  return PMP_OK;
}

Particles from_cic(const pmp_cic* p) {
  Particles P{};
  P.x = p->x; P.y = p->y; P.z = p->z; P.a = p->m;
  P.n = p->n; P.box_off = (const long long*)p->box_off;
  return P;
}
Particles from_sn(const pmp_sn* p) {
  Particles P{};
  P.x = p->x; P.y = p->y; P.z = p->z; P.b = p->m; P.c = p->e; P.r = p->r;
  P.n = p->n; P.box_off = (const long long*)p->box_off;
  return P;
}
Particles from_sinks(const pmp_sinks* p) {
  Particles P{};
  P.x = p->x; P.y = p->y; P.z = p->z; P.a = p->a;
  P.n = p->n; P.box_off = (const long long*)p->box_off;
  return P;
}

int do_deposit(pmp_ctx* c, void* buf, const void* state, const pmp_cic* cic, const pmp_sn* sn,
               const pmp_sinks* sinks, const pmp_limits* limits, hipStream_t s) {
  if (!buf) return fail(PMP_EINVAL, "buffer is NULL");
  const bool has_cic = cic && cic->n > 0;
  const bool has_sn = sn && sn->n > 0;
  const bool has_sink = sinks && sinks->n > 0;
  if (has_cic) {
    if (!cic->x || !cic->y || !cic->z || !cic->m || !cic->box_off)
      return fail(PMP_EINVAL, "CIC arrays must be non-NULL");
    if (c->ghost < 1) return fail(PMP_ERANGE, "CIC deposits need ghost width >= 1");
  }
  if (has_sn) {
    if (!sn->x || !sn->y || !sn->z || !sn->m || !sn->e || !sn->r || !sn->box_off)
      return fail(PMP_EINVAL, "supernova arrays must be non-NULL");
    if (!(sn->r_max >= 0.0) || std::floor(sn->r_max + 0.5) > c->ghost)
      return fail(PMP_ERANGE, "supernova reach floor(r_max + 1/2) exceeds ghost width %d",
                  c->ghost);
  }
  if (has_sink) {
    int rc = check_sinks(c, sinks);
    if (rc) return rc;
    if (!state) return fail(PMP_EINVAL, "sinks read the state: state is NULL");
    rc = check_limits(limits);
    if (rc) return rc;
    rc = ensure_sink_scratch(c, sinks->n, s);
    if (rc) return rc;
  }
  const Mesh M = c->mesh();
  {
    PhaseTimer t(c, PMP_PHASE_ZERO, s);
    PMP_HIP(launch_zero(buf, c->buffer_elems * (long long)c->acc_bytes(), c->tune.block, s));
  }
  if (has_cic) {
    PhaseTimer t(c, PMP_PHASE_CIC, s);
    PMP_HIP(launch_cic_direct(M, from_cic(cic), buf, nullptr, 0, c->tune.block, s));
  }
  if (has_sn) {
    PhaseTimer t(c, PMP_PHASE_SN, s);
    PMP_HIP(launch_sn_direct(M, from_sn(sn), buf, c->tune.sn_lanes, s));
  }
  if (has_sink) {
    PhaseTimer t(c, PMP_PHASE_SINK_DEPOSIT, s);
    PMP_HIP(launch_sink_deposit(M, from_sinks(sinks), state, buf, c->d_sink_scratch,
                                sinks->r_k, sinks->r_gauss, to_limits(limits), s));
  }
  return PMP_OK;
}

int do_sink_update(pmp_ctx* c, const void* state, const void* buf, const pmp_sinks* sinks,
                   const pmp_limits* limits, double* dm, double* dpx, double* dpy, double* dpz,
                   hipStream_t s) {
  if (!sinks || sinks->n == 0) return PMP_OK;
  int rc = check_sinks(c, sinks);
  if (rc) return rc;
  rc = check_limits(limits);
  if (rc) return rc;
  if (!state || !buf || !dm || !dpx || !dpy || !dpz)
    return fail(PMP_EINVAL, "sink update: NULL array");
  if (sinks->n > c->sink_cap)
    return fail(PMP_EINVAL, "sink update before a deposit with these sinks");
  PhaseTimer t(c, PMP_PHASE_SINK_UPDATE, s);
  PMP_HIP(launch_sink_update(c->mesh(), from_sinks(sinks), state, buf, c->d_sink_scratch,
                             sinks->r_k, sinks->r_gauss, to_limits(limits), dm, dpx, dpy, dpz,
                             s));
  return PMP_OK;
}

int do_apply(pmp_ctx* c, void* state, const void* buf, const pmp_limits* limits, double* eta,
             hipStream_t s) {
  if (!state || !buf) return fail(PMP_EINVAL, "apply: state or buffer is NULL");
  int rc = check_limits(limits);
  if (rc) return rc;
  PhaseTimer t(c, PMP_PHASE_APPLY, s);
  PMP_HIP(launch_apply(c->mesh(), state, buf, to_limits(limits), eta, c->tune.block, s));
  return PMP_OK;
}

int do_fold(pmp_ctx* c, void* buf, hipStream_t s) {
  PhaseTimer t(c, PMP_PHASE_FOLD, s);
  PMP_HIP(launch_fold(c->mesh(), buf, c->tune.block, s));
  return PMP_OK;
}

int do_step(pmp_ctx* c, void* state, void* buf, const pmp_cic* cic, const pmp_sn* sn,
            const pmp_sinks* sinks, const pmp_limits* limits, double* sink_out, hipStream_t s) {
  int rc = do_deposit(c, buf, state, cic, sn, sinks, limits, s);
  if (rc) return rc;
  rc = do_fold(c, buf, s);
  if (rc) return rc;
  if (sinks && sinks->n > 0) {
    if (!sink_out) return fail(PMP_EINVAL, "sinks given but sink_out is NULL");
    const long long n = sinks->n;
    rc = do_sink_update(c, state, buf, sinks, limits, sink_out, sink_out + n, sink_out + 2 * n,
                        sink_out + 3 * n, s);
    if (rc) return rc;
  }
  return do_apply(c, state, buf, limits, nullptr, s);
}

}  // namespace

extern "C" {

const char* pmp_last_error(void) { return g_last_error.c_str(); }

int pmp_create(pmp_ctx** out, const pmp_layout* L) {
  if (!out || !L) return fail(PMP_EINVAL, "pmp_create: NULL argument");
  *out = nullptr;
  if (L->nbox < 1 || !L->lo || !L->n) return fail(PMP_EINVAL, "layout needs nbox >= 1 and boxes");
  if (L->ghost < 0) return fail(PMP_EINVAL, "ghost width must be >= 0");
  if (!(L->dx > 0.0)) return fail(PMP_EINVAL, "dx must be > 0");
  if (L->acc < PMP_ACC_F32 || L->acc > PMP_ACC_FIX64) return fail(PMP_EINVAL, "bad acc type");
  if (L->state != PMP_STATE_F32 && L->state != PMP_STATE_F64)
    return fail(PMP_EINVAL, "bad state type");
  for (int a = 0; a < 3; ++a)
    if (L->domain[a] < 1) return fail(PMP_EINVAL, "domain must be >= 1 cell per axis");
  pmp_ctx* c = new (std::nothrow) pmp_ctx();
  if (!c) return fail(PMP_ENOMEM, "out of host memory");
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(PMP_EDEVICE, "no HIP device");
  }
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) ==
          hipSuccess && ncu > 0)
    c->num_cu = ncu;
  c->nbox = L->nbox;
  c->ghost = L->ghost;
  for (int a = 0; a < 3; ++a) c->domain[a] = L->domain[a];
  c->dx = L->dx;
  c->V = (L->dx * L->dx) * L->dx;
  c->acc = L->acc;
  c->state = L->state;
  c->nfield = L->with_sinks ? 6 : 5;
  c->hboxes.resize(c->nbox);
  c->dboxes.resize(c->nbox);
  std::vector<long long> owned_prefix(c->nbox + 1, 0), shell_prefix(c->nbox + 1, 0);
  long long soff = 0, boff = 0;
  for (int b = 0; b < c->nbox; ++b) {
    HostBox& h = c->hboxes[b];
    DevBox& d = c->dboxes[b];
    std::memset(&d, 0, sizeof d);
    long long ncell = 1, npad = 1;
    for (int a = 0; a < 3; ++a) {
      h.lo[a] = L->lo[3 * b + a];
      h.n[a] = L->n[3 * b + a];
      if (h.n[a] < 1 || h.lo[a] < 0 || (long long)h.lo[a] + h.n[a] > c->domain[a]) {
        delete c;
        return fail(PMP_ERANGE, "box %d outside the domain or empty", b);
      }
      d.lo[a] = h.lo[a];
      d.n[a] = h.n[a];
      d.p[a] = h.n[a] + 2 * c->ghost;
      ncell *= h.n[a];
      npad *= d.p[a];
    }
    if (ncell >= (1ll << 31)) {
      delete c;
      return fail(PMP_ERANGE, "box %d has 2^31 or more cells", b);
    }
    d.ncell = ncell;
    d.npad = npad;
    d.soff = soff;
    d.boff = boff;
    soff += 5 * ncell;
    boff += (long long)c->nfield * npad;
    owned_prefix[b + 1] = owned_prefix[b] + ncell;
    shell_prefix[b + 1] = shell_prefix[b] + shell_count(h.n, c->ghost);
  }
  c->state_elems = soff;
  c->buffer_elems = boff;
  c->owned_cells = owned_prefix[c->nbox];
  c->shell_cells = shell_prefix[c->nbox];
  // overlap check: every box against the boxes its region touches
  {
    BoxIndex idx;
    idx.build(c->hboxes, c->domain);
    for (int b = 0; b < c->nbox; ++b) {
      int lo[3], hi[3];
      for (int a = 0; a < 3; ++a) {
        lo[a] = c->hboxes[b].lo[a];
        hi[a] = lo[a] + c->hboxes[b].n[a];
      }
      bool overlap = false;
      idx.query(lo, hi, [&](int o) {
        if (o == b) return;
        bool sep = false;
        for (int a = 0; a < 3; ++a)
          if (c->hboxes[o].lo[a] >= hi[a] || c->hboxes[o].lo[a] + c->hboxes[o].n[a] <= lo[a])
            sep = true;
        if (!sep) overlap = true;
      });
      if (overlap) {
        delete c;
        return fail(PMP_ERANGE, "box %d overlaps another box", b);
      }
    }
  }
  std::vector<int> seg_off;
  std::vector<DevSeg> segs;
  build_fold_plan(c, seg_off, segs);
  c->nseg = (int)segs.size();
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = dev_alloc(&c->d_boxes, c->nbox);
  if (e == hipSuccess) e = dev_alloc(&c->d_owned_prefix, c->nbox + 1);
  if (e == hipSuccess) e = dev_alloc(&c->d_shell_prefix, c->nbox + 1);
  if (e == hipSuccess) e = dev_alloc(&c->d_seg_off, c->nbox + 1);
  if (e == hipSuccess) e = dev_alloc(&c->d_segs, segs.size());
  if (e == hipSuccess) e = dev_alloc(&c->d_status, 1);
  if (e == hipSuccess)
    e = hipMemcpy(c->d_boxes, c->dboxes.data(), sizeof(DevBox) * c->nbox, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(c->d_owned_prefix, owned_prefix.data(), sizeof(long long) * (c->nbox + 1),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(c->d_shell_prefix, shell_prefix.data(), sizeof(long long) * (c->nbox + 1),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(c->d_seg_off, seg_off.data(), sizeof(int) * (c->nbox + 1),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess && !segs.empty())
    e = hipMemcpy(c->d_segs, segs.data(), sizeof(DevSeg) * segs.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(c->d_status, 0, sizeof(DevStatus));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    release(c);
    delete c;
    return fail(PMP_EDEVICE, "pmp_create: %s", hipGetErrorString(e));
  }
  c->tune.deposit_path = 0;
  c->tune.tile = 8;
  c->tune.dense_min = 64;
  c->tune.chunk = 4096;
  c->tune.block = 256;
  c->tune.grid_per_cu = 32;
  c->tune.sn_lanes = 64;
  *out = c;
  return PMP_OK;
}

void pmp_destroy(pmp_ctx* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  release(c);
  delete c;
}

int pmp_sizes(const pmp_ctx* c, int64_t* state_elems, int64_t* buffer_elems,
              int64_t* owned_cells) {
  if (!c) return fail(PMP_EINVAL, "NULL context");
  if (state_elems) *state_elems = c->state_elems;
  if (buffer_elems) *buffer_elems = c->buffer_elems;
  if (owned_cells) *owned_cells = c->owned_cells;
  return PMP_OK;
}

int pmp_deposit(pmp_ctx* c, void* buf, const void* state, const pmp_cic* cic, const pmp_sn* sn,
                const pmp_sinks* sinks, const pmp_limits* limits, void* stream) {
  if (!c) return fail(PMP_EINVAL, "NULL context");
  return do_deposit(c, buf, state, cic, sn, sinks, limits, (hipStream_t)stream);
}

int pmp_ghost_fold(pmp_ctx* c, void* buf, void* stream) {
  if (!c || !buf) return fail(PMP_EINVAL, "NULL argument");
  return do_fold(c, buf, (hipStream_t)stream);
}

int pmp_sink_update(pmp_ctx* c, const void* state, const void* buf, const pmp_sinks* sinks,
                    const pmp_limits* limits, double* dm, double* dpx, double* dpy,
                    double* dpz, void* stream) {
  if (!c) return fail(PMP_EINVAL, "NULL context");
  return do_sink_update(c, state, buf, sinks, limits, dm, dpx, dpy, dpz, (hipStream_t)stream);
}

int pmp_apply(pmp_ctx* c, void* state, const void* buf, const pmp_limits* limits, double* eta,
              void* stream) {
  if (!c) return fail(PMP_EINVAL, "NULL context");
  return do_apply(c, state, buf, limits, eta, (hipStream_t)stream);
}

int pmp_step(pmp_ctx* c, void* state, void* buf, const pmp_cic* cic, const pmp_sn* sn,
             const pmp_sinks* sinks, const pmp_limits* limits, double* sink_out, void* stream) {
  if (!c) return fail(PMP_EINVAL, "NULL context");
  return do_step(c, state, buf, cic, sn, sinks, limits, sink_out, (hipStream_t)stream);
}

int pmp_graph_build(pmp_ctx* c, int nsteps, void* state, void* buf, const pmp_cic* cic,
                    const pmp_sn* sn, const pmp_sinks* sinks, const pmp_limits* limits,
                    double* sink_out, void* stream) {
  if (!c || nsteps < 1) return fail(PMP_EINVAL, "graph_build: bad argument");
  hipStream_t caller = (hipStream_t)stream;
  // size every scratch array before capture (no allocation inside a graph)
  if (sinks && sinks->n > 0) {
    int rc = ensure_sink_scratch(c, sinks->n, caller);
    if (rc) return rc;
  }
  if (c->graph_exec) {
    (void)hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
  }
  if (c->graph) {
    (void)hipGraphDestroy(c->graph);
    c->graph = nullptr;
  }
  PMP_HIP(hipStreamSynchronize(caller));
  hipStream_t cs;
  PMP_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return fail(PMP_EDEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  int rc = PMP_OK;
  for (int i = 0; i < nsteps && rc == PMP_OK; ++i)
    rc = do_step(c, state, buf, cic, sn, sinks, limits, sink_out, cs);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(cs, &g);
  (void)hipStreamDestroy(cs);
  if (rc != PMP_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(PMP_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(PMP_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  c->graph = g;
  c->graph_exec = ex;
  return PMP_OK;
}

int pmp_graph_launch(pmp_ctx* c, void* stream) {
  if (!c || !c->graph_exec) return fail(PMP_EINVAL, "no graph built");
  PMP_HIP(hipGraphLaunch(c->graph_exec, (hipStream_t)stream));
  return PMP_OK;
}

int pmp_get_status(pmp_ctx* c, pmp_status* out, int reset) {
  if (!c || !out) return fail(PMP_EINVAL, "NULL argument");
  PMP_HIP(hipDeviceSynchronize());
  DevStatus d;
  PMP_HIP(hipMemcpy(&d, c->d_status, sizeof d, hipMemcpyDeviceToHost));
  out->flags = d.flags;
  out->reserved = 0;
  out->touched = (int64_t)d.touched;
  out->bind = (int64_t)d.bind;
  out->lam = (int64_t)d.lam;
  out->fall = (int64_t)d.fall;
  if (reset) {
    PMP_HIP(launch_clear_status(c->d_status, nullptr));
    PMP_HIP(hipDeviceSynchronize());
  }
  return PMP_OK;
}

int pmp_get_tuning(const pmp_ctx* c, pmp_tuning* out) {
  if (!c || !out) return fail(PMP_EINVAL, "NULL argument");
  *out = c->tune;
  return PMP_OK;
}

int pmp_set_tuning(pmp_ctx* c, const pmp_tuning* t) {
  if (!c || !t) return fail(PMP_EINVAL, "NULL argument");
  if (t->deposit_path < 0 || t->deposit_path > 1) return fail(PMP_EINVAL, "deposit_path 0 or 1");
  if (t->tile != 4 && t->tile != 8 && t->tile != 16) return fail(PMP_EINVAL, "tile 4, 8 or 16");
  if (t->dense_min < 1 || t->chunk < 64) return fail(PMP_EINVAL, "dense_min >= 1, chunk >= 64");
  if (t->block != 64 && t->block != 128 && t->block != 256 && t->block != 512 &&
      t->block != 1024)
    return fail(PMP_EINVAL, "block must be 64..1024, a power of two");
  if (t->grid_per_cu < 1 || t->grid_per_cu > 64) return fail(PMP_EINVAL, "grid_per_cu 1..64");
  if (t->sn_lanes != 16 && t->sn_lanes != 32 && t->sn_lanes != 64)
    return fail(PMP_EINVAL, "sn_lanes 16, 32 or 64");
  c->tune = *t;
  return PMP_OK;
}

int pmp_autotune(pmp_ctx* c, void* state, void* buf, const pmp_cic* cic, const pmp_sn* sn,
                 const pmp_sinks* sinks, const pmp_limits* limits, double* sink_out,
                 void* stream, double* best_ms) {
  (void)c; (void)state; (void)buf; (void)cic; (void)sn; (void)sinks; (void)limits;
  (void)sink_out; (void)stream; (void)best_ms;
  return fail(PMP_EUNSUPPORTED, "autotune not built yet");
}

int pmp_profile_begin(pmp_ctx* c, int max_launches) {
  if (!c || max_launches < 1) return fail(PMP_EINVAL, "profile_begin: bad argument");
  prof_free(c);
  for (int p = 0; p < PMP_NPHASE; ++p) {
    c->prof_events[p].resize(2 * (size_t)max_launches, nullptr);
    for (auto& e : c->prof_events[p]) {
      hipError_t err = hipEventCreate(&e);
      if (err != hipSuccess) {
        e = nullptr;
        prof_free(c);
        return fail(PMP_EDEVICE, "hipEventCreate: %s", hipGetErrorString(err));
      }
    }
  }
  c->prof_max = max_launches;
  c->prof_on = true;
  return PMP_OK;
}

int pmp_profile_end(pmp_ctx* c, double* ms, int64_t* launches) {
  if (!c) return fail(PMP_EINVAL, "NULL context");
  if (!c->prof_on) return fail(PMP_EINVAL, "profiling was not started");
  PMP_HIP(hipDeviceSynchronize());
  for (int p = 0; p < PMP_NPHASE; ++p) {
    double sum = 0.0;
    for (int i = 0; i < c->prof_count[p]; ++i) {
      float t = 0.f;
      PMP_HIP(hipEventElapsedTime(&t, c->prof_events[p][2 * i], c->prof_events[p][2 * i + 1]));
      sum += t;
    }
    if (ms) ms[p] = sum;
    if (launches) launches[p] = c->prof_count[p];
  }
  prof_free(c);
  return PMP_OK;
}

int pmp_stream_copy(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src) return fail(PMP_EINVAL, "NULL argument");
  if (bytes % 4) return fail(PMP_EINVAL, "bytes must be a multiple of 4");
  PMP_HIP(launch_copy(dst, src, (long long)bytes, (hipStream_t)stream));
  return PMP_OK;
}

}  // extern "C"
