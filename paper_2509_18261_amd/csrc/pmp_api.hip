// Host side of libpmp: context, geometry checks, ghost-fold plan, HIP graph
// capture, tuning and the C-ABI entry points declared in include/pmp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pmp_internal.h"

using namespace pmp;

// Scratch of pmp_sink_create_noalloc: the creation passes' key list and rank
// accumulators (count, kCreateMax keys, kCreateMax ranks).  Every GPU the
// library runs on holds its own copy until the process ends; host code uses
// only the per-device address from hipGetSymbolAddress (noalloc_scratch).
static __device__ __align__(256) long long scratch[2 * kCreateMax + 1];

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

// Device address of `scratch` per device, looked up once per device (with
// that device current) by pmp_create.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
long long* g_scratch_ptr[kMaxDevices] = {};

int noalloc_scratch(int device, long long** out) {
  if (device < 0 || device >= kMaxDevices)
    return fail(PMP_EDEVICE, "device %d outside the scratch table (%d devices)", device,
                kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(PMP_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[device] = (long long*)p;
  }
  *out = g_scratch_ptr[device];
  return PMP_OK;
}

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
  int channels = 0;                     // PMP_CH_* bits present
  int slot[6] = {0, 1, 2, 3, 4, -1};  // buffer slot per channel, -1 absent
  std::vector<HostBox> hboxes;
  std::vector<DevBox> dboxes;
  long long state_elems = 0, buffer_elems = 0, owned_cells = 0, shell_cells = 0;
  bool tiles_domain = false;  // the boxes (disjoint, inside the domain) own every cell
  long long* noalloc_scratch = nullptr;  // this device's `scratch` (pmp_sink_create_noalloc)
  int nseg = 0;
  // device allocations
  DevBox* d_boxes = nullptr;
  long long* d_owned_prefix = nullptr;
  long long* d_shell_prefix = nullptr;
  DevStatus* d_status = nullptr;
  double* d_sink_scratch = nullptr;
  long long sink_cap = 0;
  double* d_bound = nullptr;  // reproducibility mode with sinks: error bounds [buffer_elems]
  int margin = 28;            // reproducibility mode: truncation margin M
  int num_cu = 256;
  int max_lds = 65536;  // LDS bytes one workgroup may use
  pmp_tuning tune{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  // binned deposit: tiles of the padded boxes and their scratch
  int tile_dims[3] = {0, 0, 0};
  long long ntiles = 0;
  long long* d_tile_prefix = nullptr;
  int* d_tiles_axis = nullptr;
  TileGeo* d_tile_geo = nullptr;
  // owner tiles of the same edge (fold-free step), when they fit the layout
  bool owner_ok = false;
  long long ontiles = 0;
  long long* d_otile_prefix = nullptr;
  int* d_otiles_axis = nullptr;
  TileGeo* d_otile_geo = nullptr;
  NbrBox* d_onbr = nullptr;  // [27 nbox] neighbour table on the owner grid
  BinWork bw{};
  long long bw_hist = 0, bw_blocks = 0, bw_tiles = 0, bw_nsn = 0, bw_hist2 = 0,
            bw_slice_base = 0, bw_partial = 0;
  // caller-owned workspace (pmp_set_workspace): every scratch array is carved
  // from it, sink scratch first, and nothing is allocated by the library
  char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t ws_sink_bytes = 0;  // sink scratch of the current deposit
  // phase profiler: events[phase][2 * launch + {0: start, 1: stop}]
  bool prof_on = false;
  int prof_max = 0;
  int prof_count[PMP_NPHASE] = {0};
  std::vector<hipEvent_t> prof_events[PMP_NPHASE];

  int* d_zone_off = nullptr;   // [28 nbox]
  ZoneSeg* d_zone_seg = nullptr;
  int* d_own_start = nullptr;  // owner index (multi-box layouts), see Mesh
  int* d_own_box = nullptr;
  std::vector<int> h_nbr;      // neighbour boxes per direction (owner tiles), see NbrBox
  int own_bin[3] = {1, 1, 1}, own_dims[3] = {1, 1, 1};
  int2* d_apply_chunks = nullptr;
  int2* d_fold_chunks = nullptr;
  std::vector<long long> apply_chunk_off, fold_chunk_off;  // [nbox+1] host
  Mesh mesh() const {
    Mesh M;
    M.boxes = d_boxes;
    M.all_boxes = d_boxes;
    M.nbox = nbox;
    M.ghost = ghost;
    for (int a = 0; a < 3; ++a) M.domain[a] = domain[a];
    M.V = V;
    M.nfield = nfield;
    for (int f = 0; f < 6; ++f) M.slot[f] = slot[f];
    M.acc = acc;
    M.margin = margin;
    M.state = state;
    M.buffer_elems = buffer_elems;
    M.owned_cells = owned_cells;
    M.owned_prefix = d_owned_prefix;
    M.shell_prefix = d_shell_prefix;
    M.zone_off = d_zone_off;
    M.zone_seg = d_zone_seg;
    M.apply_chunks = d_apply_chunks;
    M.n_apply_chunks = apply_chunk_off.empty() ? 0 : apply_chunk_off.back();
    M.fold_chunks = d_fold_chunks;
    M.n_fold_chunks = fold_chunk_off.empty() ? 0 : fold_chunk_off.back();
    M.shell_cells = shell_cells;
    M.status = d_status;
    M.num_cu = num_cu;
    M.own_start = d_own_start;
    M.own_box = d_own_box;
    for (int a = 0; a < 3; ++a) {
      M.own_bin[a] = own_bin[a];
      M.own_dims[a] = own_dims[a];
    }
    return M;
  }
  size_t acc_bytes() const { return acc == PMP_ACC_F32 ? 4 : 8; }
  TileGrid tiles(bool owner = false) const {
    TileGrid T;
    for (int a = 0; a < 3; ++a) {
      T.t[a] = tile_dims[a];
      T.ts[a] = __builtin_ctz((unsigned)tile_dims[a]);
    }
    T.owner = owner ? 1 : 0;
    T.tile_prefix = owner ? d_otile_prefix : d_tile_prefix;
    T.tiles_axis = owner ? d_otiles_axis : d_tiles_axis;
    T.geo = owner ? d_otile_geo : d_tile_geo;
    T.ntiles = owner ? ontiles : ntiles;
    T.gx = owner ? 0 : ghost;
    T.nbr = owner ? d_onbr : nullptr;
    T.wx = tile_dims[0] + 2 * T.gx;
    return T;
  }
};

namespace {

void free_bin_work(pmp_ctx* c) {
  BinWork& w = c->bw;
  (void)hipFree(w.hist);
  (void)hipFree(w.block_sums);
  (void)hipFree(w.cic_tmp);
  (void)hipFree(w.cic_tmp_tile);
  (void)hipFree(w.cic_rec);
  (void)hipFree(w.cic_off);
  (void)hipFree(w.sn_tmp);
  (void)hipFree(w.sn_tmp_tile);
  (void)hipFree(w.sn_rec);
  (void)hipFree(w.sn_off);
  (void)hipFree(w.sn_pk);
  (void)hipFree(w.slice_base);
  (void)hipFree(w.hist2);
  (void)hipFree(w.block_sums2);
  (void)hipFree(w.heavy_base);
  (void)hipFree(w.sink_flag);
  (void)hipFree(w.heavy_unit);
  (void)hipFree(w.heavy_count);
  (void)hipFree(w.arrive);
  (void)hipFree(w.partial);
  w = BinWork{};
  c->bw_hist = c->bw_blocks = c->bw_tiles = c->bw_nsn = c->bw_hist2 = c->bw_slice_base = 0;
  c->bw_partial = 0;
}

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
  (void)hipFree(c->d_status);
  if (!c->ws) {  // in a workspace: the caller's memory
    (void)hipFree(c->d_sink_scratch);
    (void)hipFree(c->d_bound);
  }
  (void)hipFree(c->d_tile_prefix);
  (void)hipFree(c->d_tiles_axis);
  (void)hipFree(c->d_tile_geo);
  (void)hipFree(c->d_otile_prefix);
  (void)hipFree(c->d_otiles_axis);
  (void)hipFree(c->d_otile_geo);
  (void)hipFree(c->d_zone_off);
  (void)hipFree(c->d_zone_seg);
  (void)hipFree(c->d_own_start);
  (void)hipFree(c->d_own_box);
  (void)hipFree(c->d_onbr);
  (void)hipFree(c->d_apply_chunks);
  (void)hipFree(c->d_fold_chunks);
  if (!c->ws) free_bin_work(c);
}

// Owner tiles of edge (tx, tyz, tyz) need every tile extent along an axis to
// be at most domain - 2g cells (a stencil then meets one periodic image of a
// tile at most, and never two images of one cell).
bool owner_tiles_fit(const pmp_ctx* c, int tx, int tyz) {
  const int t[3] = {tx, tyz, tyz};
  for (int a = 0; a < 3; ++a) {
    int widest = 0;
    for (int b = 0; b < c->nbox; ++b) widest = std::max(widest, std::min(t[a], c->dboxes[b].n[a]));
    if (widest > c->domain[a] - 2 * c->ghost) return false;
  }
  return true;
}

// Tiles of edge (tx, tyz, tyz): over every padded box, or (owner) over the
// owned cells of every box.
struct HostGrid {
  std::vector<long long> prefix;
  std::vector<int> axis;
  std::vector<TileGeo> geo;
};

int make_grid(const pmp_ctx* c, int tx, int tyz, bool owner, HostGrid& H) {
  const int t[3] = {tx, tyz, tyz};
  const int g0 = c->ghost;
  H.prefix.assign(c->nbox + 1, 0);
  H.axis.assign(3 * (size_t)c->nbox, 0);
  for (int b = 0; b < c->nbox; ++b) {
    // the tile pass indexes a tile's cells by 32-bit offsets from its origin
    const DevBox& db = c->dboxes[b];
    if ((long long)db.p[0] * db.p[1] * tyz >= (1ll << 31))
      return fail(PMP_ERANGE, "box %d: %d padded planes of %d x %d cells reach 2^31; use tile_yz < %d",
                  b, tyz, db.p[0], db.p[1], tyz);
    long long n = 1;
    for (int a = 0; a < 3; ++a) {
      const int p = db.p[a];
      // x: boundaries on owned cells g + k t (first and last take the ghosts)
      H.axis[3 * b + a] =
          (a == 0 || owner) ? (db.n[a] + t[a] - 1) / t[a] : (p + t[a] - 1) / t[a];
      n *= H.axis[3 * b + a];
    }
    H.prefix[b + 1] = H.prefix[b] + n;
  }
  if (2 * H.prefix[c->nbox] + 1 >= (1ll << 31))
    return fail(PMP_ERANGE, "too many tiles (%lld); use larger tiles", H.prefix[c->nbox]);
  // per-tile geometry, in tile order (x fastest within a box)
  H.geo.assign((size_t)H.prefix[c->nbox], TileGeo{});
  for (int b = 0; b < c->nbox; ++b) {
    const DevBox& d = c->dboxes[b];
    const int* ax = &H.axis[3 * (size_t)b];
    long long q = H.prefix[b];
    for (int tz = 0; tz < ax[2]; ++tz)
      for (int ty = 0; ty < ax[1]; ++ty)
        for (int tx_ = 0; tx_ < ax[0]; ++tx_, ++q) {
          TileGeo& G = H.geo[(size_t)q];
          std::memset(&G, 0, sizeof G);
          const int tc[3] = {tx_, ty, tz};
          G.boff = d.boff;
          G.soff = d.soff;
          G.b = b;
          for (int a = 0; a < 3; ++a) {
            G.p[a] = d.p[a];
            if (owner) {
              // owned cells [tc t, (tc + 1) t) of the box; padded-local origin
              G.o[a] = g0 + tc[a] * t[a];
              G.ext[a] = std::min(t[a], d.n[a] - tc[a] * t[a]);
            } else if (a == 0) {
              G.o[0] = (tx_ == 0) ? 0 : g0 + tx_ * t[0];
              const int end = (tx_ == ax[0] - 1) ? d.p[0] : g0 + (tx_ + 1) * t[0];
              G.ext[0] = end - G.o[0];
            } else {
              G.o[a] = tc[a] * t[a];
              G.ext[a] = std::min(t[a], d.p[a] - G.o[a]);
            }
            G.glo[a] = G.o[a] - g0 + d.lo[a];
          }
        }
  }
  return PMP_OK;
}

int upload_grid(const HostGrid& H, long long** dp, int** da, TileGeo** dt) {
  *dp = nullptr;
  *da = nullptr;
  *dt = nullptr;
  hipError_t e = dev_alloc(dp, H.prefix.size());
  if (e == hipSuccess) e = dev_alloc(da, H.axis.size());
  if (e == hipSuccess) e = dev_alloc(dt, std::max<size_t>(H.geo.size(), 1));
  if (e == hipSuccess)
    e = hipMemcpy(*dp, H.prefix.data(), sizeof(long long) * H.prefix.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(*da, H.axis.data(), sizeof(int) * H.axis.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !H.geo.empty())
    e = hipMemcpy(*dt, H.geo.data(), sizeof(TileGeo) * H.geo.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(*dp);
    (void)hipFree(*da);
    (void)hipFree(*dt);
    return fail(PMP_EDEVICE, "tile grid: %s", hipGetErrorString(e));
  }
  return PMP_OK;
}

// Both tile grids for edge (tx, tyz, tyz); the owner grid only where owner
// tiles fit the layout.
int build_tiles(pmp_ctx* c, int tx, int tyz) {
  HostGrid H, O;
  if (int rc = make_grid(c, tx, tyz, false, H)) return rc;
  const bool own = owner_tiles_fit(c, tx, tyz);
  if (own)
    if (int rc = make_grid(c, tx, tyz, true, O)) return rc;
  long long* dp = nullptr;
  int* da = nullptr;
  TileGeo* dt = nullptr;
  long long* op = nullptr;
  int* oa = nullptr;
  TileGeo* ot = nullptr;
  NbrBox* on = nullptr;
  if (int rc = upload_grid(H, &dp, &da, &dt)) return rc;
  if (own) {
    int rc = upload_grid(O, &op, &oa, &ot);
    if (!rc) {
      // the neighbour table with each neighbour's owner tiles
      std::vector<NbrBox> nb(27 * (size_t)c->nbox);
      for (size_t q = 0; q < nb.size(); ++q) {
        NbrBox& R = nb[q];
        std::memset(&R, 0, sizeof R);
        R.id = c->h_nbr[q];
        if (R.id < 0) continue;
        const DevBox& d = c->dboxes[R.id];
        for (int a = 0; a < 3; ++a) {
          R.lo[a] = d.lo[a];
          R.n[a] = d.n[a];
          R.tax[a] = O.axis[3 * (size_t)R.id + a];
        }
        R.tprefix = (int)O.prefix[R.id];
      }
      hipError_t e = dev_alloc(&on, nb.size());
      if (e == hipSuccess)
        e = hipMemcpy(on, nb.data(), sizeof(NbrBox) * nb.size(), hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        (void)hipFree(on);
        (void)hipFree(op);
        (void)hipFree(oa);
        (void)hipFree(ot);
        rc = fail(PMP_EDEVICE, "neighbour table: %s", hipGetErrorString(e));
      }
    }
    if (rc) {
      (void)hipFree(dp);
      (void)hipFree(da);
      (void)hipFree(dt);
      return rc;
    }
  }
  (void)hipFree(c->d_tile_prefix);
  (void)hipFree(c->d_tiles_axis);
  (void)hipFree(c->d_tile_geo);
  (void)hipFree(c->d_otile_prefix);
  (void)hipFree(c->d_otiles_axis);
  (void)hipFree(c->d_otile_geo);
  (void)hipFree(c->d_onbr);
  c->d_onbr = on;
  c->d_tile_prefix = dp;
  c->d_tiles_axis = da;
  c->d_tile_geo = dt;
  c->d_otile_prefix = op;
  c->d_otiles_axis = oa;
  c->d_otile_geo = ot;
  c->owner_ok = own;
  for (int a = 0; a < 3; ++a) c->tile_dims[a] = tx;
  c->tile_dims[1] = c->tile_dims[2] = tyz;
  c->ntiles = H.prefix[c->nbox];
  c->ontiles = own ? O.prefix[c->nbox] : 0;
  return PMP_OK;
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

// Zone lists: per box and per zone (3 x 3 x 3 split of each axis into
// [0, g), [g, n - g), [n - g, n)), the plan's segments that reach the zone, in
// plan order.  A shell cell only tests the segments of its own zone.
void build_zones(const pmp_ctx* c, const std::vector<int>& seg_off,
                 const std::vector<DevSeg>& segs, std::vector<int>& zone_off,
                 std::vector<ZoneSeg>& zone_seg) {
  zone_off.assign(28 * (size_t)c->nbox, 0);
  zone_seg.clear();
  for (int b = 0; b < c->nbox; ++b) {
    int zl[3][3], zh[3][3];
    for (int a = 0; a < 3; ++a) {
      const int n = c->hboxes[b].n[a];
      const int gl = std::min(c->ghost, n), hs = std::max(gl, n - c->ghost);
      zl[a][0] = 0;  zh[a][0] = gl;
      zl[a][1] = gl; zh[a][1] = hs;
      zl[a][2] = hs; zh[a][2] = n;
    }
    for (int z = 0; z < 27; ++z) {
      zone_off[28 * (size_t)b + z] = (int)zone_seg.size();
      const int zz[3] = {z % 3, (z / 3) % 3, z / 9};
      for (int q = seg_off[b]; q < seg_off[b + 1]; ++q) {
        bool hit = true;
        for (int a = 0; a < 3; ++a) {
          const int l = std::max(segs[q].lo[a], zl[a][zz[a]]);
          const int h = std::min(segs[q].hi[a], zh[a][zz[a]]);
          if (l >= h) hit = false;
        }
        if (hit) {
          const DevSeg& S = segs[q];
          const DevBox& src = c->dboxes[S.src];
          ZoneSeg Z;
          for (int a = 0; a < 3; ++a) {
            Z.lo[a] = S.lo[a];
            Z.hi[a] = S.hi[a];
          }
          Z.p0 = src.p[0];
          Z.p1 = src.p[1];
          Z.base = src.boff + ((long long)S.off[2] * src.p[1] + S.off[1]) * src.p[0] + S.off[0];
          Z.npad = src.npad;
          zone_seg.push_back(Z);
        }
      }
    }
    zone_off[28 * (size_t)b + 27] = (int)zone_seg.size();
  }
}

// Chunks of kChunk cells per box for counts[b] cells; off[b] is box b's first chunk.
void build_chunks(const std::vector<long long>& counts, std::vector<int2>& chunks,
                  std::vector<long long>& off) {
  chunks.clear();
  off.assign(counts.size() + 1, 0);
  for (size_t b = 0; b < counts.size(); ++b) {
    for (long long c0 = 0; c0 < counts[b]; c0 += kChunk) chunks.push_back(make_int2((int)b, (int)c0));
    off[b + 1] = (long long)chunks.size();
  }
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
  return st == hipStreamCaptureStatusActive;
}

size_t sink_scratch_bytes(long long n);

// Bytes of the error bounds the reproducibility mode keeps for the sinks'
// global-atomic deposit (one per buffer element), 256-byte aligned.
size_t bound_bytes(const pmp_ctx* c) {
  return c->acc == PMP_ACC_F64R ? ((size_t)c->buffer_elems * 8 + 255) & ~(size_t)255 : 0;
}

int ensure_sink_scratch(pmp_ctx* c, long long n, hipStream_t s) {
  if (c->ws) {
    const size_t sb = sink_scratch_bytes(n), need = sb + bound_bytes(c);
    if (need > c->ws_bytes)
      return fail(PMP_ERANGE, "workspace of %zu bytes is too small for %lld sinks", c->ws_bytes, n);
    c->d_sink_scratch = reinterpret_cast<double*>(c->ws);
    c->d_bound = bound_bytes(c) ? reinterpret_cast<double*>(c->ws + sb) : nullptr;
    c->sink_cap = n;
    c->ws_sink_bytes = need;
    return PMP_OK;
  }
  if (bound_bytes(c) && !c->d_bound) {
    if (capturing(s)) return fail(PMP_EINVAL, "sink scratch must be sized before graph capture");
    PMP_HIP(dev_alloc(&c->d_bound, (size_t)c->buffer_elems));
  }
  if (n <= c->sink_cap) return PMP_OK;
  if (capturing(s))
    return fail(PMP_EINVAL, "sink scratch must be sized before graph capture");
  (void)hipFree(c->d_sink_scratch);
  c->d_sink_scratch = nullptr;
  c->sink_cap = 0;
  PMP_HIP(dev_alloc(&c->d_sink_scratch, (size_t)(kSinkScratch * n)));
  c->sink_cap = n;
  return PMP_OK;
}

// Most tiles a cell range of `len` cells can touch along an axis of tile edge t.
long long tiles_for(long long len, int t) { return (len + t - 1) / t + 1; }

// Size the binned-deposit scratch for these particle counts (never while a
// graph is being captured).  Record arrays are sized for the most tiles a
// particle can touch (8 for CIC; for a sphere, from its largest reach).
template <class T> int regrow(T** p, long long have, long long need) {
  if (need <= have) return PMP_OK;
  (void)hipFree(*p);
  *p = nullptr;
  PMP_HIP(dev_alloc(p, (size_t)need));
  return PMP_OK;
}

// Sizes (elements) of the binned-deposit scratch arrays for these particle
// counts and the current tiles.
struct BinSizes {
  int shift = 0, nb = 0;
  long long hist = 0, blocks = 0, tiles1 = 0, partial = 0, slot_cap = 0, cic_cap = 0,
            sn_cap = 0, hist2 = 0, blocks2 = 0, slice_base = 0, n_sn = 0;
};

// The step runs on owner tiles (no ghost zone, no fold): tuning fuse_apply 2
// where the owner tiles fit the layout, the binned path, no reproducibility
// mode.  (Steps with sinks never do.)
bool owner_step(const pmp_ctx* c) {
  return c->tune.fuse_apply == 2 && c->owner_ok && c->tune.deposit_path == 1 &&
         c->acc != PMP_ACC_F64R;
}

int bin_sizes(const pmp_ctx* c, long long n_cic, long long n_sn, double r_max, BinSizes& z) {
  const int* t = c->tile_dims;
  const long long span = 2 * (long long)std::ceil(std::max(r_max, 0.0)) + 3;
  long long maxt = tiles_for(span, t[0]) * tiles_for(span, t[1]) * tiles_for(span, t[2]);
  if (owner_step(c)) {
    // owner tiles: per axis the span splits into segments at box faces and
    // at the periodic wrap, each adding at most two tiles (never more tiles
    // than cells)
    long long m = 1;
    for (int a = 0; a < 3; ++a) {
      long long seg = 2;
      if (c->nbox > 1 || c->d_own_start) {
        int edge = c->domain[a];
        for (const auto& b : c->hboxes) edge = std::min(edge, b.n[a]);
        seg = (span - 1) / std::max(edge, 1) + 2;
      }
      m *= std::min<long long>(span, (span + t[a] - 1) / t[a] + 2 * seg - 1);
    }
    maxt = std::max(maxt, m);
  }
  const long long nbc = (n_cic + kBinChunkCic - 1) / kBinChunkCic;
  const long long nbs = (n_sn + kBinChunkSn - 1) / kBinChunkSn;
  const long long cic_cap = std::max<long long>(8 * n_cic, 1);
  const long long sn_cap = std::max<long long>(maxt * n_sn, 1);
  const long long full_slices = (cic_cap + kSlice - 1) / kSlice + (sn_cap + kSlice - 1) / kSlice;
  // coarse buckets of 2^shift consecutive tiles (at most 1024 buckets, at
  // most 8192 tiles per bucket; sized for the padded grid, which never has
  // fewer tiles than the owner grid): the shift that minimises the histogram work,
  // level 1 (nb x blocks counts, written one cache line apart, weighted 4)
  // plus level 2 (2^shift x slices counts, zeroed and scanned)
  int shift = -1;
  double best = 0.0;
  for (int sh = 0; sh <= 13; ++sh) {
    const long long nbs_ = (c->ntiles + (1ll << sh) - 1) >> sh;
    if (nbs_ > 1024) continue;
    const double cost = 4.0 * (double)nbs_ * (double)(nbc + nbs) +
                        (double)(1ll << sh) * (double)(full_slices + 2 * nbs_);
    if (shift < 0 || cost < best) {
      shift = sh;
      best = cost;
    }
  }
  if (shift < 0) return fail(PMP_ERANGE, "binned deposit: too many tiles (%lld)", c->ntiles);
  z.shift = shift;
  z.nb = (int)((c->ntiles + (1ll << shift) - 1) >> shift);
  z.hist = (long long)z.nb * (nbc + nbs) + 1;
  z.blocks = (z.hist + 1023) / 1024 + 1;
  z.tiles1 = c->ntiles + 1;
  // every bucket can add one partial slice to the full ones
  const long long max_slices = full_slices + 2 * (long long)z.nb;
  z.hist2 = (max_slices << shift) + 1;
  z.blocks2 = (z.hist2 + 1023) / 1024 + 1;
  // chunk slots for split tiles, each holding two channels of a padded LDS tile
  z.slot_cap = 4ll * c->num_cu;
  z.partial = z.slot_cap * 2 * (long long)(t[0] + 2 * c->ghost + 1) * t[1] * t[2];
  z.cic_cap = cic_cap;
  z.sn_cap = sn_cap;
  z.slice_base = 2 * (long long)z.nb + 1;
  z.n_sn = std::max<long long>(n_sn, 1);
  if (cic_cap >= (1ll << 31) || sn_cap >= (1ll << 31) || z.hist >= (1ll << 31) ||
      z.hist2 >= (1ll << 31))
    return fail(PMP_ERANGE, "binned deposit: too many tile entries");
  return PMP_OK;
}

// The scratch arrays laid out one after another from base, each 256-byte
// aligned; returns the bytes used.  With w non-null, w's arrays point there.
size_t carve_bin(const BinSizes& z, char* base, BinWork* w) {
  size_t off = 0;
  BinWork tmp{};
  BinWork& W = w ? *w : tmp;
  auto take = [&](auto*& p, long long count) {
    using T = typename std::remove_reference<decltype(*p)>::type;
    off = (off + 255) & ~(size_t)255;
    p = reinterpret_cast<T*>(base + off);
    off += (size_t)std::max<long long>(count, 1) * sizeof(T);
  };
  double* partial = nullptr;
  take(W.hist, z.hist);
  take(W.block_sums, z.blocks);
  take(W.cic_off, z.tiles1);
  take(W.sn_off, z.tiles1);
  take(W.heavy_base, z.tiles1);
  take(W.sink_flag, z.tiles1);
  take(partial, z.partial);
  W.partial = partial;
  take(W.heavy_unit, z.slot_cap);
  take(W.arrive, z.slot_cap);
  take(W.heavy_count, 1);
  take(W.cic_tmp, z.cic_cap);
  take(W.cic_tmp_tile, z.cic_cap);
  take(W.cic_rec, z.cic_cap);
  take(W.sn_tmp, z.sn_cap);
  take(W.sn_tmp_tile, z.sn_cap);
  take(W.sn_rec, z.sn_cap);
  take(W.hist2, z.hist2);
  take(W.block_sums2, z.blocks2);
  take(W.slice_base, z.slice_base);
  take(W.sn_pk, z.n_sn);
  if (w) {
    W.cic_cap = z.cic_cap;
    W.sn_cap = z.sn_cap;
    W.slot_cap = z.slot_cap;
    W.shift = z.shift;
    W.nbuckets = z.nb;
    W.max_slices = (z.hist2 - 1) >> z.shift;
  }
  return off;
}

size_t sink_scratch_bytes(long long n) {
  return ((size_t)std::max<long long>(kSinkScratch * n, 1) * sizeof(double) + 255) &
         ~(size_t)255;
}

int ensure_bin_work(pmp_ctx* c, long long n_cic, long long n_sn, double r_max, hipStream_t s) {
  BinSizes z;
  if (int rc = bin_sizes(c, n_cic, n_sn, r_max, z)) return rc;
  if (c->ws) {
    // caller-owned workspace: carve, after the sink scratch of this deposit
    const size_t need = c->ws_sink_bytes + carve_bin(z, nullptr, nullptr);
    if (need > c->ws_bytes)
      return fail(PMP_ERANGE, "workspace of %zu bytes is too small: this deposit needs %zu",
                  c->ws_bytes, need);
    carve_bin(z, c->ws + c->ws_sink_bytes, &c->bw);
    return PMP_OK;
  }
  const int shift = z.shift, nb = z.nb;
  const long long hist = z.hist, blocks = z.blocks, hist2 = z.hist2, blocks2 = z.blocks2;
  const long long slot_cap = z.slot_cap, partial = z.partial, cic_cap = z.cic_cap,
                  sn_cap = z.sn_cap;
  c->bw.shift = shift;
  c->bw.nbuckets = nb;
  const bool grow = hist > c->bw_hist || blocks > c->bw_blocks || c->ntiles + 1 > c->bw_tiles ||
                    cic_cap > c->bw.cic_cap || sn_cap > c->bw.sn_cap || n_sn > c->bw_nsn ||
                    hist2 > c->bw_hist2 || 2 * nb + 1 > c->bw_slice_base ||
                    partial > c->bw_partial;
  // launches are sized by this deposit's slices, not by the scratch's
  // capacity (which keeps the largest size seen)
  c->bw.max_slices = (hist2 - 1) >> shift;
  if (!grow) return PMP_OK;
  if (capturing(s)) return fail(PMP_EINVAL, "binned-deposit scratch must be sized before capture");
  PMP_HIP(hipStreamSynchronize(s));
  BinWork& w = c->bw;
  int rc = PMP_OK;
  if (!rc && hist > c->bw_hist) {
    rc = regrow(&w.hist, 0, hist);
    if (!rc) c->bw_hist = hist;
  }
  if (!rc && blocks > c->bw_blocks) {
    rc = regrow(&w.block_sums, 0, blocks);
    if (!rc) c->bw_blocks = blocks;
  }
  if (!rc && c->ntiles + 1 > c->bw_tiles) {
    rc = regrow(&w.cic_off, 0, c->ntiles + 1);
    if (!rc) rc = regrow(&w.sn_off, 0, c->ntiles + 1);
    if (!rc) rc = regrow(&w.heavy_base, 0, c->ntiles + 1);
    if (!rc) rc = regrow(&w.sink_flag, 0, c->ntiles + 1);
    if (!rc) c->bw_tiles = c->ntiles + 1;
  }
  if (!rc && partial > c->bw_partial) {
    rc = regrow(reinterpret_cast<double**>(&w.partial), 0, partial);
    if (!rc && !w.heavy_unit) rc = regrow(&w.heavy_unit, 0, slot_cap);
    if (!rc && !w.arrive) rc = regrow(&w.arrive, 0, slot_cap);
    if (!rc && !w.heavy_count) rc = regrow(&w.heavy_count, 0, 1);
    if (!rc) {
      w.slot_cap = slot_cap;
      c->bw_partial = partial;
    }
  }
  if (!rc && cic_cap > w.cic_cap) {
    rc = regrow(&w.cic_tmp, 0, cic_cap);
    if (!rc) rc = regrow(&w.cic_tmp_tile, 0, cic_cap);
    if (!rc) rc = regrow(&w.cic_rec, 0, cic_cap);
    if (!rc) w.cic_cap = cic_cap;
  }
  if (!rc && sn_cap > w.sn_cap) {
    rc = regrow(&w.sn_tmp, 0, sn_cap);
    if (!rc) rc = regrow(&w.sn_tmp_tile, 0, sn_cap);
    if (!rc) rc = regrow(&w.sn_rec, 0, sn_cap);
    if (!rc) w.sn_cap = sn_cap;
  }
  if (!rc && hist2 > c->bw_hist2) {
    rc = regrow(&w.hist2, 0, hist2);
    if (!rc) rc = regrow(&w.block_sums2, 0, blocks2);
    if (!rc) c->bw_hist2 = hist2;
  }
  if (!rc && 2 * nb + 1 > c->bw_slice_base) {
    rc = regrow(&w.slice_base, 0, 2 * (long long)nb + 1);
    if (!rc) c->bw_slice_base = 2 * nb + 1;
  }
  if (!rc && n_sn > c->bw_nsn) {
    rc = regrow(&w.sn_pk, 0, n_sn);
    if (!rc) c->bw_nsn = n_sn;
  }
  if (rc) free_bin_work(c);  // a failed allocation leaves no half-sized scratch behind
  return rc;
}

Limits to_limits(const pmp_ctx* c, const pmp_limits* L) {
  Limits l;
  l.rho_floor = L->rho_floor;
  l.rho_tr = L->rho_tr;
  l.cap = L->cap;
  l.eint_mode = L->eint_mode;
  l.truelove_J = L->truelove_J;
  l.G = L->G;
  l.gamma = L->gamma;
  l.dx = c->dx;
  return l;
}

int check_limits(const pmp_limits* L) {
  if (!L) return fail(PMP_EINVAL, "limits is NULL");
  if (!(L->cap >= 0.0) || !(L->rho_floor >= 0.0) || std::isnan(L->rho_tr))
    return fail(PMP_EINVAL, "bad limits (cap %g, rho_floor %g, rho_tr %g)", L->cap,
                L->rho_floor, L->rho_tr);
  if (L->eint_mode != 0 && L->eint_mode != 1)
    return fail(PMP_EINVAL, "eint_mode must be 0 or 1");
  if (std::isnan(L->truelove_J) || !std::isfinite(L->truelove_J))
    return fail(PMP_EINVAL, "truelove_J must be finite");
  if (L->truelove_J > 0.0 && (!(L->G > 0.0) || !std::isfinite(L->G) || !(L->gamma >= 1.0) ||
                              !std::isfinite(L->gamma)))
    return fail(PMP_EINVAL, "a per-cell Truelove density needs finite G > 0 and gamma >= 1");
  return PMP_OK;
}

bool covers_domain(const pmp_ctx* c) {
  if (c->nbox != 1) return false;
  for (int a = 0; a < 3; ++a)
    if (c->hboxes[0].lo[a] != 0 || c->hboxes[0].n[a] != c->domain[a]) return false;
  return true;
}

// Owner index for kernels that read cells of other boxes (the sinks): bins
// of the smallest box extent per axis (at least domain / 128, so the index
// stays small), each listing the boxes that overlap it.  With bins no larger
// than any box, a bin meets at most two boxes per axis.
void build_owner_index(pmp_ctx* c, std::vector<int>& start, std::vector<int>& boxes) {
  for (int a = 0; a < 3; ++a) {
    int m = c->domain[a];
    for (const auto& b : c->hboxes) m = std::min(m, b.n[a]);
    m = std::max(m, (c->domain[a] + 127) / 128);
    c->own_bin[a] = std::max(m, 1);
    c->own_dims[a] = (c->domain[a] + c->own_bin[a] - 1) / c->own_bin[a];
  }
  const size_t nbin = (size_t)c->own_dims[0] * c->own_dims[1] * c->own_dims[2];
  std::vector<std::vector<int>> bins(nbin);
  for (int i = 0; i < c->nbox; ++i) {
    const HostBox& b = c->hboxes[i];
    int b0[3], b1[3];
    for (int a = 0; a < 3; ++a) {
      b0[a] = b.lo[a] / c->own_bin[a];
      b1[a] = (b.lo[a] + b.n[a] - 1) / c->own_bin[a];
    }
    for (int z = b0[2]; z <= b1[2]; ++z)
      for (int y = b0[1]; y <= b1[1]; ++y)
        for (int x = b0[0]; x <= b1[0]; ++x)
          bins[((size_t)z * c->own_dims[1] + y) * c->own_dims[0] + x].push_back(i);
  }
  start.assign(nbin + 1, 0);
  for (size_t q = 0; q < nbin; ++q) start[q + 1] = start[q] + (int)bins[q].size();
  boxes.clear();
  boxes.reserve(start[nbin]);
  for (const auto& v : bins) boxes.insert(boxes.end(), v.begin(), v.end());
}

// Neighbour table for owner tiles (see Mesh::nbr): for every box and each of
// the 27 directions, the boxes whose owned cells meet the region next to the
// box in that direction, found through the box index over the region's
// periodic pieces.
void build_neighbour_table(const pmp_ctx* c, std::vector<int>& nbr) {
  const int g = c->ghost;
  BoxIndex idx;
  idx.build(c->hboxes, c->domain);
  nbr.assign(27 * (size_t)c->nbox, -1);
  for (int b = 0; b < c->nbox; ++b) {
    const HostBox& B = c->hboxes[b];
    for (int d = 0; d < 27; ++d) {
      const int dir[3] = {d % 3 - 1, (d / 3) % 3 - 1, d / 9 - 1};
      // the region per axis, then its pieces inside [0, D)
      int pl[3][2], ph[3][2], np[3];
      bool empty = false;
      for (int a = 0; a < 3; ++a) {
        const int D = c->domain[a];
        int r0, r1;
        if (dir[a] < 0) { r0 = B.lo[a] - g; r1 = B.lo[a] - 1; }
        else if (dir[a] > 0) { r0 = B.lo[a] + B.n[a]; r1 = B.lo[a] + B.n[a] + g - 1; }
        else { r0 = B.lo[a]; r1 = B.lo[a] + B.n[a] - 1; }
        if (r1 < r0) { empty = true; break; }
        if (r1 - r0 + 1 >= D) { pl[a][0] = 0; ph[a][0] = D - 1; np[a] = 1; continue; }
        const int l = ((r0 % D) + D) % D, h = l + (r1 - r0);
        if (h < D) { pl[a][0] = l; ph[a][0] = h; np[a] = 1; }
        else { pl[a][0] = l; ph[a][0] = D - 1; pl[a][1] = 0; ph[a][1] = h - D; np[a] = 2; }
      }
      if (empty) continue;
      int found = -1, count = 0;
      for (int cz = 0; cz < np[2]; ++cz)
        for (int cy = 0; cy < np[1]; ++cy)
          for (int cx = 0; cx < np[0]; ++cx) {
            const int lo[3] = {pl[0][cx], pl[1][cy], pl[2][cz]};
            const int hi[3] = {ph[0][cx] + 1, ph[1][cy] + 1, ph[2][cz] + 1};
            idx.query(lo, hi, [&](int q) {
              const HostBox& Q = c->hboxes[q];
              for (int a = 0; a < 3; ++a)
                if (Q.lo[a] >= hi[a] || Q.lo[a] + Q.n[a] <= lo[a]) return;
              if (q != found) {
                found = q;
                ++count;
              }
            });
          }
      // (a box met through two pieces counts once: pieces are visited one
      // after another, so a repeat of the last box found is not counted)
      nbr[27 * (size_t)b + d] = count == 0 ? -1 : (count == 1 ? found : -2);
    }
  }
}

int check_sinks(const pmp_ctx* c, const pmp_sinks* k) {
  if (k->rate != PMP_SINK_FRACTION && k->rate != PMP_SINK_BONDI)
    return fail(PMP_EINVAL, "sink rate %d is not a pmp_sink_rate_t", (int)k->rate);
  if (!k->x || !k->y || !k->z || !k->box_off || (k->rate == PMP_SINK_FRACTION && !k->a))
    return fail(PMP_EINVAL, "sink arrays must be non-NULL");
  if (k->rate == PMP_SINK_BONDI) {
    if (!k->m || !k->vx || !k->vy || !k->vz)
      return fail(PMP_EINVAL, "Bondi-Hoyle sinks need the mass and velocity arrays");
    if (!(k->r_k >= 0.5))
      return fail(PMP_EINVAL, "Bondi-Hoyle sinks need r_k >= 1/2 (r_acc in [1/4, r_k/2])");
    if (!(k->G >= 0.0) || !std::isfinite(k->G) || !(k->dt >= 0.0) || !std::isfinite(k->dt) ||
        !(k->gamma >= 1.0) || !std::isfinite(k->gamma) || !(k->lambda >= 0.0) ||
        !std::isfinite(k->lambda))
      return fail(PMP_EINVAL, "Bondi-Hoyle sinks need finite G, dt, lambda >= 0, gamma >= 1");
  }
  if (c->slot[5] < 0)
    return fail(PMP_EINVAL, "sinks need a layout with the removal channel K (with_sinks = 1)");
  if (!(k->r_k >= 0.0) || (k->rate == PMP_SINK_FRACTION && !(k->r_gauss > 0.0)))
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

SinkParams sink_params(const pmp_ctx* c, const pmp_sinks* p) {
  SinkParams K{};
  K.m = p->m; K.vx = p->vx; K.vy = p->vy; K.vz = p->vz;
  K.r_k = p->r_k; K.r_gauss = p->r_gauss; K.dx = c->dx;
  K.G = p->G; K.dt = p->dt; K.gamma = p->gamma; K.lambda = p->lambda;
  K.rate = p->rate;
  return K;
}

// fuse_state non-null: the binned path also applies the interior cells (a
// step without sinks), or, on owner tiles (owner), every owned cell, except,
// in a step with sinks, the tiles a sink kernel may reach: those are stored,
// the sinks add to their owning cells, and they are applied after the sink
// update.  On owner tiles without fuse_state the tile pass stores every
// owned cell.  No fold is needed on owner tiles.  *fused tells what was done
// (0: a ghost-zoned buffer to fold, 1: the interior cells applied, 2: every
// cell applied, 3: owned cells complete, 4: every cell applied but those of
// the flagged tiles, which are complete).
int do_deposit(pmp_ctx* c, void* buf, const void* state, const pmp_cic* cic, const pmp_sn* sn,
               const pmp_sinks* sinks, const pmp_limits* limits, hipStream_t s,
               void* fuse_state = nullptr, int* fused = nullptr, bool owner = false) {
  if (fused) *fused = 0;
  if (!buf) return fail(PMP_EINVAL, "buffer is NULL");
  c->ws_sink_bytes = 0;  // a workspace holds this deposit's sink scratch first, if any
  const bool has_cic = cic && cic->n > 0;
  const bool has_sn = sn && sn->n > 0;
  const bool has_sink = sinks && sinks->n > 0;
  if (has_cic) {
    if (!cic->x || !cic->y || !cic->z || !cic->m || !cic->box_off)
      return fail(PMP_EINVAL, "CIC arrays must be non-NULL");
    if (c->ghost < 1) return fail(PMP_ERANGE, "CIC deposits need ghost width >= 1");
    if (c->slot[0] < 0) return fail(PMP_EINVAL, "CIC deposits need the rho channel");
  }
  if (has_sn) {
    if (!sn->x || !sn->y || !sn->z || !sn->m || !sn->e || !sn->r || !sn->box_off)
      return fail(PMP_EINVAL, "supernova arrays must be non-NULL");
    if (!(sn->r_max >= 0.0) || std::floor(sn->r_max + 0.5) > c->ghost)
      return fail(PMP_ERANGE, "supernova reach floor(r_max + 1/2) exceeds ghost width %d",
                  c->ghost);
    if (c->slot[0] < 0 || c->slot[4] < 0)
      return fail(PMP_EINVAL, "supernova deposits need the rho and E channels");
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
  // owner tiles need the binned path (with no particles to bin, the zero
  // fill and the fold stand)
  owner = owner && c->tune.deposit_path == 1 && (has_cic || has_sn);
  if (c->tune.deposit_path == 1 && (has_cic || has_sn)) {
    int rc = ensure_bin_work(c, has_cic ? cic->n : 0, has_sn ? sn->n : 0,
                             has_sn ? sn->r_max : 0.0, s);
    if (rc) return rc;
    const Particles pc = has_cic ? from_cic(cic) : Particles{};
    const Particles ps = has_sn ? from_sn(sn) : Particles{};
    const TileGrid T = c->tiles(owner);
    const bool flagged = owner && has_sink && fuse_state;
    {
      PhaseTimer t(c, PMP_PHASE_BIN, s);
      PMP_HIP(launch_bin(M, T, has_cic ? &pc : nullptr, has_sn ? &ps : nullptr, c->bw,
                         c->tune.count_lanes, s));
      PMP_HIP(launch_tile_prep(M, T, has_cic ? &pc : nullptr, has_sn ? &ps : nullptr, c->bw,
                               c->tune, s));
      if (flagged)
        PMP_HIP(launch_sink_tiles(M, T, from_sinks(sinks), sinks->r_k, c->bw.sink_flag, s));
    }
    {
      PhaseTimer t(c, PMP_PHASE_TILE, s);
      Limits L{};
      if (fuse_state) {
        const int rc2 = check_limits(limits);
        if (rc2) return rc2;
        L = to_limits(c, limits);
      }
      PMP_HIP(launch_tile_deposit(M, T, has_cic ? &pc : nullptr, has_sn ? &ps : nullptr, c->bw,
                                  buf, c->tune, fuse_state, L, s,
                                  flagged ? c->bw.sink_flag : nullptr));
      if (fused) *fused = owner ? (fuse_state ? (flagged ? 4 : 2) : 3) : (fuse_state ? 1 : 0);
    }
  } else {
    {
      PhaseTimer t(c, PMP_PHASE_ZERO, s);
      PMP_HIP(launch_zero(buf, c->buffer_elems * (long long)c->acc_bytes(), c->tune.block, s));
    }
    if (has_cic) {
      PhaseTimer t(c, PMP_PHASE_CIC, s);
      PMP_HIP(launch_cic_direct(M, from_cic(cic), buf, c->tune.block, s));
    }
    if (has_sn) {
      PhaseTimer t(c, PMP_PHASE_SN, s);
      PMP_HIP(launch_sn_direct(M, from_sn(sn), buf, c->tune.sn_lanes, s));
    }
  }
  if (has_sink) {
    PhaseTimer t(c, PMP_PHASE_SINK_DEPOSIT, s);
    SinkParams K = sink_params(c, sinks);
    K.owner = owner ? 1 : 0;
    PMP_HIP(launch_sink_deposit(M, from_sinks(sinks), state, buf, c->d_sink_scratch, K,
                                to_limits(c, limits), c->d_bound, s));
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
                             sink_params(c, sinks), to_limits(c, limits), dm, dpx, dpy, dpz,
                             s));
  return PMP_OK;
}

int do_apply(pmp_ctx* c, void* state, const void* buf, const pmp_limits* limits, double* eta,
             hipStream_t s) {
  if (!state || !buf) return fail(PMP_EINVAL, "apply: state or buffer is NULL");
  int rc = check_limits(limits);
  if (rc) return rc;
  PhaseTimer t(c, PMP_PHASE_APPLY, s);
  PMP_HIP(launch_apply(c->mesh(), state, buf, to_limits(c, limits), eta, c->tune.block, s));
  return PMP_OK;
}

int do_fold(pmp_ctx* c, void* buf, hipStream_t s) {
  PhaseTimer t(c, PMP_PHASE_FOLD, s);
  PMP_HIP(launch_fold(c->mesh(), buf, c->tune.block, s));
  return PMP_OK;
}

int do_step(pmp_ctx* c, void* state, void* buf, const pmp_cic* cic, const pmp_sn* sn,
            const pmp_sinks* sinks, const pmp_limits* limits, double* sink_out, hipStream_t s) {
  const bool has_sinks = sinks && sinks->n > 0;
  const bool owner = owner_step(c);
  int fused = 0;
  int rc = do_deposit(c, buf, state, cic, sn, sinks, limits, s,
                      ((!has_sinks && c->tune.fuse_apply) || owner) && state ? state : nullptr,
                      &fused, owner);
  if (rc) return rc;
  if (fused == 2) return PMP_OK;  // owner tiles: every owned cell is done
  if (fused == 1) {
    // interior cells are done; fold and apply the shell
    PhaseTimer t(c, PMP_PHASE_FOLD, s);
    PMP_HIP(launch_fold_apply(c->mesh(), state, buf, to_limits(c, limits), s));
    return PMP_OK;
  }
  if (fused != 3 && fused != 4) {  // owner tiles hold every contribution in the owned cells
    rc = do_fold(c, buf, s);
    if (rc) return rc;
  }
  if (sinks && sinks->n > 0) {
    if (!sink_out) return fail(PMP_EINVAL, "sinks given but sink_out is NULL");
    const long long n = sinks->n;
    rc = do_sink_update(c, state, buf, sinks, limits, sink_out, sink_out + n, sink_out + 2 * n,
                        sink_out + 3 * n, s);
    if (rc) return rc;
  }
  if (fused == 4) {
    // owner tiles with sinks: the tiles a sink kernel may reach, now
    PhaseTimer t(c, PMP_PHASE_APPLY, s);
    PMP_HIP(launch_apply_tiles(c->mesh(), c->tiles(true), state, buf, c->bw.sink_flag,
                               to_limits(c, limits), s));
    return PMP_OK;
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
  if (L->ghost < 0 || L->ghost > 64) return fail(PMP_EINVAL, "ghost width must be 0..64");
  if (!(L->dx > 0.0)) return fail(PMP_EINVAL, "dx must be > 0");
  if (L->acc < PMP_ACC_F32 || L->acc > PMP_ACC_F64R) return fail(PMP_EINVAL, "bad acc type");
  if (L->acc == PMP_ACC_F64R && (L->margin_bits < 0 || L->margin_bits > 52))
    return fail(PMP_EINVAL, "margin_bits must be 0 .. 52");
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
  if (noalloc_scratch(c->device, &c->noalloc_scratch) != PMP_OK) {
    delete c;
    return PMP_EDEVICE;
  }
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) ==
          hipSuccess && ncu > 0)
    c->num_cu = ncu;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) ==
          hipSuccess && lds > 0)
    c->max_lds = lds;
  c->nbox = L->nbox;
  c->ghost = L->ghost;
  for (int a = 0; a < 3; ++a) c->domain[a] = L->domain[a];
  c->dx = L->dx;
  c->V = (L->dx * L->dx) * L->dx;
  c->acc = L->acc;
  c->margin = L->margin_bits;
  c->state = L->state;
  {
    const int all = PMP_CH_RHO | PMP_CH_MOM | PMP_CH_E | PMP_CH_K;
    int ch = L->channels;
    if (ch == 0) ch = PMP_CH_RHO | PMP_CH_MOM | PMP_CH_E | (L->with_sinks ? PMP_CH_K : 0);
    if (ch & ~all) {
      delete c;
      return fail(PMP_EINVAL, "channels 0x%x has unknown bits", L->channels);
    }
    if ((ch & PMP_CH_MOM) != 0 && (ch & PMP_CH_MOM) != PMP_CH_MOM) {
      delete c;
      return fail(PMP_EINVAL, "the momentum channels come together (PMP_CH_MOM)");
    }
    if (L->with_sinks ? !(ch & PMP_CH_K) : (ch & PMP_CH_K) != 0) {
      delete c;
      return fail(PMP_EINVAL, "PMP_CH_K is present exactly when with_sinks = 1");
    }
    c->channels = ch;
    c->nfield = 0;
    for (int f = 0; f < 6; ++f) c->slot[f] = (ch >> f) & 1 ? c->nfield++ : -1;
    if (c->nfield == 0) {
      delete c;
      return fail(PMP_EINVAL, "layout has no buffer channel");
    }
  }
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
  c->tiles_domain =
      c->owned_cells == (long long)c->domain[0] * c->domain[1] * (long long)c->domain[2];
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
  std::vector<int> zone_off;
  std::vector<ZoneSeg> zone_seg;
  build_zones(c, seg_off, segs, zone_off, zone_seg);
  std::vector<long long> owned_counts(c->nbox), shell_counts(c->nbox);
  for (int b = 0; b < c->nbox; ++b) {
    owned_counts[b] = owned_prefix[b + 1] - owned_prefix[b];
    shell_counts[b] = shell_prefix[b + 1] - shell_prefix[b];
    c->dboxes[b].shell = (int)shell_counts[b];
  }
  std::vector<int2> apply_chunks, fold_chunks;
  build_chunks(owned_counts, apply_chunks, c->apply_chunk_off);
  build_chunks(shell_counts, fold_chunks, c->fold_chunk_off);
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = dev_alloc(&c->d_boxes, c->nbox);
  if (e == hipSuccess) e = dev_alloc(&c->d_owned_prefix, c->nbox + 1);
  if (e == hipSuccess) e = dev_alloc(&c->d_shell_prefix, c->nbox + 1);
  if (e == hipSuccess) e = dev_alloc(&c->d_status, 1);
  if (e == hipSuccess)
    e = hipMemcpy(c->d_boxes, c->dboxes.data(), sizeof(DevBox) * c->nbox, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(c->d_owned_prefix, owned_prefix.data(), sizeof(long long) * (c->nbox + 1),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(c->d_shell_prefix, shell_prefix.data(), sizeof(long long) * (c->nbox + 1),
                  hipMemcpyHostToDevice);
  auto upload = [&](auto** dst, const auto& v) {
    if (e == hipSuccess) e = dev_alloc(dst, v.size());
    if (e == hipSuccess && !v.empty())
      e = hipMemcpy(*dst, v.data(), sizeof(v[0]) * v.size(), hipMemcpyHostToDevice);
  };
  upload(&c->d_zone_off, zone_off);
  upload(&c->d_zone_seg, zone_seg);
  if (!covers_domain(c)) {
    std::vector<int> own_start, own_box;
    build_owner_index(c, own_start, own_box);
    upload(&c->d_own_start, own_start);
    upload(&c->d_own_box, own_box);
  }
  upload(&c->d_apply_chunks, apply_chunks);
  upload(&c->d_fold_chunks, fold_chunks);
  if (e == hipSuccess) e = hipMemset(c->d_status, 0, sizeof(DevStatus));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    release(c);
    delete c;
    return fail(PMP_EDEVICE, "pmp_create: %s", hipGetErrorString(e));
  }
  c->tune.deposit_path = 1;
  c->tune.tile_x = 64;
  c->tune.tile_yz = 4;
  c->tune.tile_block = 256;
  c->tune.block = 256;
  c->tune.grid_per_cu = 32;
  c->tune.sn_lanes = 64;
  c->tune.tile_grid_per_cu = 0;
  c->tune.chunk_cic = 4096;
  c->tune.chunk_sn = 512;
  c->tune.fuse_apply = 1;
  c->tune.count_lanes = 4;
  build_neighbour_table(c, c->h_nbr);
  {
    int rc = build_tiles(c, c->tune.tile_x, c->tune.tile_yz);
    if (rc) {
      release(c);
      delete c;
      return rc;
    }
  }
  *out = c;
  return PMP_OK;
}

void pmp_destroy(pmp_ctx* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  release(c);
  delete c;
}

int pmp_workspace_size(const pmp_ctx* c, int64_t max_cic, int64_t max_sn, double max_sn_radius,
                       int64_t max_sinks, size_t* bytes) {
  if (!c || !bytes) return fail(PMP_EINVAL, "NULL argument");
  if (max_cic < 0 || max_sn < 0 || max_sinks < 0 || !(max_sn_radius >= 0.0))
    return fail(PMP_EINVAL, "workspace_size: negative count or radius");
  size_t total = max_sinks > 0 ? sink_scratch_bytes(max_sinks) + bound_bytes(c) : 0;
  if (max_cic > 0 || max_sn > 0) {
    BinSizes z;
    if (int rc = bin_sizes(c, max_cic, max_sn, max_sn_radius, z)) return rc;
    total += carve_bin(z, nullptr, nullptr);
  }
  *bytes = std::max<size_t>((total + 255) & ~(size_t)255, 256);
  return PMP_OK;
}

int pmp_set_workspace(pmp_ctx* c, void* dev_ptr, size_t bytes) {
  if (!c) return fail(PMP_EINVAL, "NULL context");
  if (dev_ptr && ((uintptr_t)dev_ptr & 255))
    return fail(PMP_EINVAL, "workspace must be 256-byte aligned");
  if (dev_ptr && bytes < 256) return fail(PMP_EINVAL, "workspace smaller than 256 bytes");
  if (c->graph_exec)
    return fail(PMP_EINVAL, "a built graph holds scratch addresses: set the workspace first");
  PMP_HIP(hipDeviceSynchronize());
  // the library's own scratch is released, or, leaving a workspace, forgotten
  if (!c->ws) {
    free_bin_work(c);
    (void)hipFree(c->d_sink_scratch);
    (void)hipFree(c->d_bound);
  } else {
    c->bw = BinWork{};
  }
  c->d_sink_scratch = nullptr;
  c->d_bound = nullptr;
  c->sink_cap = 0;
  c->ws = static_cast<char*>(dev_ptr);
  c->ws_bytes = dev_ptr ? bytes : 0;
  c->ws_sink_bytes = 0;
  return PMP_OK;
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

int pmp_deposit_snr(pmp_ctx* c, void* buf, const void* state, const pmp_snr* snr,
                    double* info, void* stream) {
  if (!c) return fail(PMP_EINVAL, "NULL context");
  if (!buf || !state || !snr) return fail(PMP_EINVAL, "buffer, state and remnants must be non-NULL");
  if (c->acc == PMP_ACC_F64R)
    return fail(PMP_EUNSUPPORTED, "supernova remnants: not in the reproducibility mode");
  if (snr->n < 0) return fail(PMP_EINVAL, "supernova remnants: negative count");
  if (snr->n == 0) return PMP_OK;
  if (!snr->x || !snr->y || !snr->z || !snr->m || !snr->e || !snr->vx || !snr->vy || !snr->vz ||
      !snr->box_off)
    return fail(PMP_EINVAL, "supernova remnant arrays must be non-NULL");
  if (!(snr->r_k >= 0.0) || !(snr->r_k <= 16.0)) return fail(PMP_EINVAL, "r_k must lie in [0, 16]");
  if (snr->sub < 1 || snr->sub > 16 || (snr->sub & (snr->sub - 1)) != 0)
    return fail(PMP_EINVAL, "sub must be 1, 2, 4, 8 or 16");
  if (!(snr->nh_per_rho > 0.0) || !(snr->msf_coef > 0.0) || !(snr->psnr_coef >= 0.0) ||
      !(snr->eps_k >= 0.0) || !std::isfinite(snr->nh_per_rho) || !std::isfinite(snr->msf_coef) ||
      !std::isfinite(snr->psnr_coef) || !std::isfinite(snr->eps_k))
    return fail(PMP_EINVAL, "bad remnant parameters (nh_per_rho, msf_coef > 0; psnr_coef, eps_k >= 0)");
  for (int f = 0; f < 5; ++f)
    if (c->slot[f] < 0)
      return fail(PMP_EINVAL, "supernova remnants need the rho, momentum and E channels");
  if (std::floor(snr->r_k + 1.0 - 0.5 / snr->sub) > c->ghost)
    return fail(PMP_ERANGE, "remnant kernel reach exceeds the ghost width %d", c->ghost);
  SnrArgs A{};
  A.x = snr->x; A.y = snr->y; A.z = snr->z; A.m = snr->m; A.e = snr->e;
  A.vx = snr->vx; A.vy = snr->vy; A.vz = snr->vz;
  A.n = snr->n;
  A.box_off = (const long long*)snr->box_off;
  A.r_k = snr->r_k; A.sub = snr->sub;
  A.nh_per_rho = snr->nh_per_rho; A.msf_coef = snr->msf_coef;
  A.psnr_coef = snr->psnr_coef; A.eps_k = snr->eps_k;
  PhaseTimer t(c, PMP_PHASE_SNR, (hipStream_t)stream);
  PMP_HIP(launch_snr_deposit(c->mesh(), A, state, buf, info, (hipStream_t)stream));
  return PMP_OK;
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

}  // extern "C"

namespace {

// Argument checks shared by the two sink creation entry points; E receives
// the existing sinks' positions.
int create_checks(const pmp_ctx* c, const void* state, const pmp_sinks* existing, double r_k,
                  const pmp_limits* limits, int64_t max_new, const double* out, SinkPos& E) {
  if (!c) return fail(PMP_EINVAL, "NULL context");
  if (!state) return fail(PMP_EINVAL, "state is NULL");
  if (max_new < 0 || max_new > kCreateMax)
    return fail(PMP_EINVAL, "max_new must lie in [0, %lld]", (long long)kCreateMax);
  if (max_new > 0 && !out) return fail(PMP_EINVAL, "out is NULL");
  if (!(r_k >= 0.0) || !(r_k <= 16.0)) return fail(PMP_EINVAL, "r_k must lie in [0, 16]");
  int rc = check_limits(limits);
  if (rc) return rc;
  E = SinkPos{};
  if (existing && existing->n != 0) {
    if (existing->n < 0) return fail(PMP_EINVAL, "existing sinks: negative count");
    if (!existing->x || !existing->y || !existing->z)
      return fail(PMP_EINVAL, "existing sinks: position arrays must be non-NULL");
    E.x = existing->x;
    E.y = existing->y;
    E.z = existing->z;
    E.n = existing->n;
  }
  if (!c->tiles_domain)
    return fail(PMP_ERANGE, "sink creation needs boxes that tile the periodic domain");
  for (int a = 0; a < 3; ++a)
    if (std::floor(r_k) > c->domain[a])
      return fail(PMP_EINVAL, "r_k = %g reaches past the domain (%d cells along axis %d)", r_k,
                  c->domain[a], a);
  return PMP_OK;
}

}  // namespace

extern "C" {

int pmp_sink_create(pmp_ctx* c, void* state, const void* buf, const pmp_sinks* existing,
                    double r_k, const pmp_limits* limits, int64_t max_new, double* out,
                    int64_t* work, void* stream) {
  SinkPos E;
  int rc = create_checks(c, state, existing, r_k, limits, max_new, out, E);
  if (rc) return rc;
  if (!work) return fail(PMP_EINVAL, "work is NULL");
  PMP_HIP(launch_sink_create(c->mesh(), state, buf, E, r_k, to_limits(c, limits),
                             (long long)max_new, out, (long long*)work, (hipStream_t)stream));
  return PMP_OK;
}

int pmp_sink_create_noalloc(pmp_ctx* c, void* state, const void* buf,
                            const pmp_sinks* existing, double r_k, const pmp_limits* limits,
                            int64_t max_new, double* out, int64_t* count, void* stream) {
  SinkPos E;
  int rc = create_checks(c, state, existing, r_k, limits, max_new, out, E);
  if (rc) return rc;
  if (!count) return fail(PMP_EINVAL, "count is NULL");
  if (!c->noalloc_scratch) return fail(PMP_EDEVICE, "no scratch address for this device");
  hipStream_t s = (hipStream_t)stream;
  long long* work = c->noalloc_scratch;  // count, keys, ranks (2 kCreateMax + 1)
  PMP_HIP(launch_sink_create(c->mesh(), state, buf, E, r_k, to_limits(c, limits),
                             (long long)max_new, out, work, s));
  PMP_HIP(hipMemcpyAsync(count, work, sizeof(long long), hipMemcpyDeviceToDevice, s));
  return PMP_OK;
}

int pmp_step(pmp_ctx* c, void* state, void* buf, const pmp_cic* cic, const pmp_sn* sn,
             const pmp_sinks* sinks, const pmp_limits* limits, double* sink_out, void* stream) {
  if (!c) return fail(PMP_EINVAL, "NULL context");
  return do_step(c, state, buf, cic, sn, sinks, limits, sink_out, (hipStream_t)stream);
}

int pmp_step_per_box(pmp_ctx* c, void* state, void* buf, const pmp_cic* cic, const pmp_sn* sn,
                     const pmp_limits* limits, const int64_t* cic_off, const int64_t* sn_off,
                     void* stream) {
  if (!c || !state || !buf) return fail(PMP_EINVAL, "per-box step: NULL argument");
  if (c->acc == PMP_ACC_F64R)
    return fail(PMP_EINVAL, "per-box step: the reproducibility mode runs on the binned path");
  hipStream_t s = (hipStream_t)stream;
  const bool has_cic = cic && cic->n > 0, has_sn = sn && sn->n > 0;
  if (has_cic && !cic_off) return fail(PMP_EINVAL, "per-box step: cic_off (host) is NULL");
  if (has_sn && !sn_off) return fail(PMP_EINVAL, "per-box step: sn_off (host) is NULL");
  if (has_cic && c->ghost < 1) return fail(PMP_ERANGE, "CIC deposits need ghost width >= 1");
  if (has_sn && (!(sn->r_max >= 0.0) || std::floor(sn->r_max + 0.5) > c->ghost))
    return fail(PMP_ERANGE, "supernova reach exceeds the ghost width");
  int rc = check_limits(limits);
  if (rc) return rc;
  const Mesh all = c->mesh();
  const Limits L = to_limits(c, limits);
  const size_t ab = c->acc_bytes();
  // Step 1 for every box, then Step 2 for every box (the fold reads other
  // boxes' ghosts), then Steps 3 + 5 for every box.
  for (int b = 0; b < c->nbox; ++b) {
    Mesh M = all;
    M.boxes = c->d_boxes + b;
    M.nbox = 1;
    char* base = (char*)buf;
    const DevBox& D = c->dboxes[b];
    PMP_HIP(launch_zero(base + D.boff * ab, (long long)(c->nfield * D.npad) * (long long)ab,
                        c->tune.block, s));
    if (has_cic && cic_off[b + 1] > cic_off[b]) {
      Particles P = from_cic(cic);
      const long long o = cic_off[b];
      P.x += o; P.y += o; P.z += o; P.a += o;
      P.n = cic_off[b + 1] - o;
      PMP_HIP(launch_cic_direct(M, P, buf, c->tune.block, s));
    }
    if (has_sn && sn_off[b + 1] > sn_off[b]) {
      Particles P = from_sn(sn);
      const long long o = sn_off[b];
      P.x += o; P.y += o; P.z += o; P.b += o; P.c += o; P.r += o;
      P.n = sn_off[b + 1] - o;
      PMP_HIP(launch_sn_direct(M, P, buf, c->tune.sn_lanes, s));
    }
  }
  for (int b = 0; b < c->nbox; ++b) {
    Mesh M = all;
    M.fold_chunks = c->d_fold_chunks + c->fold_chunk_off[b];
    M.n_fold_chunks = c->fold_chunk_off[b + 1] - c->fold_chunk_off[b];
    PMP_HIP(launch_fold(M, buf, c->tune.block, s));
  }
  for (int b = 0; b < c->nbox; ++b) {
    Mesh M = all;
    M.apply_chunks = c->d_apply_chunks + c->apply_chunk_off[b];
    M.n_apply_chunks = c->apply_chunk_off[b + 1] - c->apply_chunk_off[b];
    PMP_HIP(launch_apply(M, state, buf, L, nullptr, c->tune.block, s));
  }
  return PMP_OK;
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
  if (c->tune.deposit_path == 1) {
    const long long nc = cic ? cic->n : 0, ns = sn ? sn->n : 0;
    int rc = ensure_bin_work(c, nc, ns, (sn && sn->n > 0) ? sn->r_max : 0.0, caller);
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
  auto pow2_in = [](int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; };
  if (t->deposit_path < 0 || t->deposit_path > 1) return fail(PMP_EINVAL, "deposit_path 0 or 1");
  if (c->acc == PMP_ACC_F64R && t->deposit_path != 1)
    return fail(PMP_EINVAL, "the reproducibility mode runs on the binned path (deposit_path 1)");
  if (!pow2_in(t->tile_x, 16, 256)) return fail(PMP_EINVAL, "tile_x must be 16, 32, 64, 128 or 256");
  if (!pow2_in(t->tile_yz, 2, 8)) return fail(PMP_EINVAL, "tile_yz must be 2, 4 or 8");
  if (!pow2_in(t->tile_block, 64, 1024)) return fail(PMP_EINVAL, "tile_block 64..1024, power of 2");
  if (!pow2_in(t->block, 64, 1024)) return fail(PMP_EINVAL, "block 64..1024, power of 2");
  if (t->grid_per_cu < 1 || t->grid_per_cu > 64) return fail(PMP_EINVAL, "grid_per_cu 1..64");
  if (t->sn_lanes != 16 && t->sn_lanes != 32 && t->sn_lanes != 64)
    return fail(PMP_EINVAL, "sn_lanes 16, 32 or 64");
  if (t->tile_grid_per_cu < 0 || t->tile_grid_per_cu > 64)
    return fail(PMP_EINVAL, "tile_grid_per_cu 0..64");
  if (t->chunk_cic < 64 || t->chunk_cic > (1 << 24)) return fail(PMP_EINVAL, "chunk_cic 64..2^24");
  if (t->chunk_sn < 16 || t->chunk_sn > (1 << 24)) return fail(PMP_EINVAL, "chunk_sn 16..2^24");
  if (t->fuse_apply < 0 || t->fuse_apply > 2) return fail(PMP_EINVAL, "fuse_apply 0, 1 or 2");
  if (t->count_lanes != 1 && t->count_lanes != 2 && t->count_lanes != 4 && t->count_lanes != 8 &&
      t->count_lanes != 16)
    return fail(PMP_EINVAL, "count_lanes 1, 2, 4, 8 or 16");
  {
    const long long lds =
        tile_lds_bytes(t->tile_x, t->tile_yz, c->ghost, c->acc == PMP_ACC_F64R);
    if (lds > c->max_lds)
      return fail(PMP_EINVAL, "tile %d x %d x %d needs %lld B of LDS, more than the %d B available",
                  t->tile_x, t->tile_yz, t->tile_yz, lds, c->max_lds);
  }
  if (t->tile_x != c->tile_dims[0] || t->tile_yz != c->tile_dims[1]) {
    if (c->graph_exec) return fail(PMP_EINVAL, "changing tiles would invalidate the built graph");
    PMP_HIP(hipDeviceSynchronize());
    int rc = build_tiles(c, t->tile_x, t->tile_yz);
    if (rc) return rc;
  }
  c->tune = *t;
  return PMP_OK;
}

int pmp_autotune(pmp_ctx* c, void* state, void* buf, const pmp_cic* cic, const pmp_sn* sn,
                 const pmp_sinks* sinks, const pmp_limits* limits, double* sink_out,
                 void* stream, double* best_ms) {
  if (!c || !state || !buf) return fail(PMP_EINVAL, "autotune: NULL argument");
  if (c->graph_exec) return fail(PMP_EINVAL, "autotune would invalidate the built graph");
  hipStream_t s = (hipStream_t)stream;
  const bool has_sn = sn && sn->n > 0;
  // candidates: the direct path and a set of tile shapes for the binned path
  std::vector<pmp_tuning> cand;
  const pmp_tuning base = c->tune;
  const bool has_sinks = sinks && sinks->n > 0;
  auto add = [&](int path, int tx, int tyz, int tb, int lanes, int tgrid, int fuse) {
    pmp_tuning t = base;
    t.deposit_path = path;
    t.tile_x = tx;
    t.tile_yz = tyz;
    t.tile_block = tb;
    t.sn_lanes = lanes;
    t.tile_grid_per_cu = tgrid;
    t.fuse_apply = fuse;
    cand.push_back(t);
  };
  add(0, base.tile_x, base.tile_yz, base.tile_block, 64, 0, 0);
  if (has_sn) add(0, base.tile_x, base.tile_yz, base.tile_block, 16, 0, 0);
  const int shapes[][3] = {{64, 4, 128}, {64, 4, 256}, {32, 4, 128}, {32, 8, 256},
                           {16, 8, 256}, {64, 2, 128}, {16, 4, 128}, {32, 4, 256},
                           {64, 8, 256}, {64, 8, 512}, {128, 4, 256}, {128, 4, 512},
                           {256, 4, 256}, {256, 4, 512}, {256, 2, 256}};
  // the interior-fused apply (1) only applies to steps without sinks; owner
  // tiles (2) wherever they fit the layout
  for (int fuse = 2; fuse >= 0; --fuse)
    for (const auto& sh : shapes) {
      if (fuse == 1 && has_sinks) continue;
      if (fuse == 2 && (c->acc == PMP_ACC_F64R || !owner_tiles_fit(c, sh[0], sh[1]))) continue;
      add(1, sh[0], sh[1], sh[2], 64, 0, fuse);
    }
  // the caller's state is left as it was: candidates run on a copy
  const size_t sbytes = (size_t)c->state_elems * (c->state == PMP_STATE_F32 ? 4 : 8);
  void* work = nullptr;
  PMP_HIP(hipMalloc(&work, sbytes));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = PMP_OK;
  double best = 1e300;
  pmp_tuning best_t = base;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    rc = fail(PMP_EDEVICE, "autotune: hipEventCreate failed");
  // time one candidate (2 warm steps, 5 timed); a shape this device cannot
  // run (LDS) is skipped
  auto time_one = [&](const pmp_tuning& cand_t) {
    if (rc != PMP_OK || pmp_set_tuning(c, &cand_t) != PMP_OK) return;
    if (c->ws && cand_t.deposit_path == 1) {
      // a caller's workspace: skip tile shapes whose scratch does not fit it
      size_t need = 0;
      if (pmp_workspace_size(c, cic ? cic->n : 0, sn ? sn->n : 0,
                             (sn && sn->n > 0) ? sn->r_max : 0.0, sinks ? sinks->n : 0,
                             &need) != PMP_OK ||
          need > c->ws_bytes)
        return;
    }
    if (launch_copy(work, state, (long long)sbytes, s) != hipSuccess) {
      rc = fail(PMP_EDEVICE, "autotune: state copy failed");
      return;
    }
    for (int w = 0; w < 2 && rc == PMP_OK; ++w)
      rc = do_step(c, work, buf, cic, sn, sinks, limits, sink_out, s);
    if (rc) return;
    const int reps = 5;
    if (hipEventRecord(e0, s) != hipSuccess) {
      rc = fail(PMP_EDEVICE, "event");
      return;
    }
    for (int r = 0; r < reps && rc == PMP_OK; ++r)
      rc = do_step(c, work, buf, cic, sn, sinks, limits, sink_out, s);
    if (rc) return;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      rc = fail(PMP_EDEVICE, "autotune: event timing failed");
      return;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double per = ms / reps;
    if (per < best) {
      best = per;
      best_t = cand_t;
    }
  };
  // stage 1: path, tile shape, workgroup size, fused apply; the list is
  // timed twice, forwards then backwards, and each candidate keeps its better
  // time (a single timing of the best shape was now and then slow enough to
  // lose to a shape 8% slower)
  for (size_t i = 0; i < cand.size() && rc == PMP_OK; ++i) time_one(cand[i]);
  for (size_t i = cand.size(); i-- > 0 && rc == PMP_OK;) time_one(cand[i]);
  // stage 2, binned path: the split thresholds (clustered inputs) and the
  // persistent grid cap, around the stage-1 winner
  if (rc == PMP_OK && best_t.deposit_path == 1) {
    const pmp_tuning w1 = best_t;
    const int chunks[][2] = {{1024, 128}, {16384, 2048}};
    for (const auto& ch : chunks) {
      pmp_tuning t = w1;
      t.chunk_cic = ch[0];
      t.chunk_sn = ch[1];
      time_one(t);
    }
    const int grids[] = {4, 16};
    const pmp_tuning w2 = best_t;
    for (int gpc : grids) {
      pmp_tuning t = w2;
      t.tile_grid_per_cu = gpc;
      time_one(t);
    }
    if (has_sn) {
      // lanes per supernova in the member count (large spheres want more)
      const pmp_tuning w3 = best_t;
      for (int lanes : {1, 2, 4, 8, 16}) {
        if (lanes == w3.count_lanes) continue;
        pmp_tuning t = w3;
        t.count_lanes = lanes;
        time_one(t);
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  (void)hipFree(work);
  const int rc2 = pmp_set_tuning(c, rc == PMP_OK ? &best_t : &base);
  if (rc) return rc;
  if (rc2) return rc2;
  if (best_ms) *best_ms = best;
  return PMP_OK;
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

int pmp_copy_bench(void* dst, const void* src, size_t bytes, int variant, void* stream) {
  if (!dst || !src) return fail(PMP_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  if (variant == 0) {
    if (bytes % 4) return fail(PMP_EINVAL, "bytes must be a multiple of 4");
    PMP_HIP(launch_copy(dst, src, (long long)bytes, s));
  } else if (variant == 1) {
    if (bytes % 16384 || ((uintptr_t)dst | (uintptr_t)src) % 16)
      return fail(PMP_EINVAL, "variant 1: bytes a multiple of 16384, 16-byte aligned pointers");
    PMP_HIP(launch_copy4(dst, src, (long long)bytes, s));
  } else if (variant == 2) {
    PMP_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
  } else {
    return fail(PMP_EINVAL, "copy variant must be 0, 1 or 2");
  }
  return PMP_OK;
}

int pmp_atomic_bench(void* dst, int64_t slots, int type, int pattern, int64_t n_ops,
                     void* stream) {
  if (!dst) return fail(PMP_EINVAL, "dst is NULL");
  if (slots < 1 || (slots & (slots - 1)) != 0)
    return fail(PMP_EINVAL, "slots must be a power of two");
  if (type < 0 || type > 2 || pattern < 0 || pattern > 2 || n_ops < 0)
    return fail(PMP_EINVAL, "type and pattern must lie in [0, 2], n_ops >= 0");
  if (n_ops == 0) return PMP_OK;
  PMP_HIP(launch_atomic_bench(dst, (long long)slots, type, pattern, (long long)n_ops,
                              (hipStream_t)stream));
  return PMP_OK;
}

}  // extern "C"
