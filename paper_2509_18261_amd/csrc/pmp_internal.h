// Internal declarations shared by the kernels (pmp_kernels.hip) and the host
// API (pmp_api.hip).  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pmp.h"

namespace pmp {

constexpr int kChunk = 256;  // cells per apply / fold work chunk (= threads per block)

// One box of the layout, in device memory.
struct DevBox {
  int lo[3];        // first owned global cell
  int n[3];         // owned cells per axis
  int p[3];         // padded cells per axis (n + 2g)
  int shell;        // owned cells within g of a face
  long long soff;   // element offset of field 0 in the state
  long long boff;   // element offset of field 0 in the buffer
  long long ncell;  // owned cells (state field stride)
  long long npad;   // padded cells (buffer field stride)
};

// One rectangle of the ghost-fold plan: owned cells [lo, hi) of the
// destination box (local owned coordinates) receive the ghost cells of box
// src at padded local index (owned local index + off).
struct DevSeg {
  int src;
  int lo[3];
  int hi[3];
  int off[3];
};

// A fold segment as one zone lists it: the destination range and the source
// addressing folded in, so that the ghost image of owned cell (i, j, k) is
// buffer element base + (k p1 + j) p0 + i (field stride npad).
struct alignas(16) ZoneSeg {
  int lo[3], hi[3];  // owned cells [lo, hi) of the destination box
  int p0, p1;        // padded extents of the source box
  long long base;    // source boff + ((off_z p1) + off_y) p0 + off_x
  long long npad;    // padded cells of the source box
};

// Device status word and counters (mirrors pmp_status).
struct DevStatus {
  unsigned int flags;
  unsigned int reserved;
  unsigned long long touched, bind, lam, fall;
};

// Limiter parameters (pmp_limits) and the cell edge.  truelove_J > 0: each
// cell's Truelove density from its own sound speed (truelove_rho).
struct Limits {
  double rho_floor, rho_tr, cap;
  int eint_mode;
  double truelove_J, G, gamma, dx;
};

// Everything a launch needs about the mesh.
struct Mesh {
  const DevBox* boxes;      // boxes this launch covers (all, or one for per-box launches)
  const DevBox* all_boxes;  // every box (fold sources)
  int nbox;
  int ghost;
  int domain[3];
  double V;
  int nfield;   // buffer channels present
  int slot[6];  // buffer slot of rho, px, py, pz, E, K, or -1 when absent
  int acc;    // pmp_acc_t
  int margin; // PMP_ACC_F64R: truncation margin M (bits)
  int state;  // pmp_state_t
  long long buffer_elems;
  long long owned_cells;
  const long long* owned_prefix;  // [nbox+1] cumulative owned cells
  const long long* shell_prefix;  // [nbox+1] cumulative shell cells
  // Each box splits along every axis into [0, g), [g, n - g), [n - g, n) (27
  // zones); zone_off[28 b + z] .. zone_off[28 b + z + 1] index zone_seg, the
  // segments (in plan order) that reach zone z of box b, with their source
  // addressing.
  const int* zone_off;
  const ZoneSeg* zone_seg;
  // Work chunks of kChunk cells that never cross a box: (global box, first
  // cell) for the apply (owned cells) and for the fold (shell cells).
  const int2* apply_chunks;
  long long n_apply_chunks;
  const int2* fold_chunks;
  long long n_fold_chunks;
  long long shell_cells;
  DevStatus* status;
  int num_cu;
  // Owner index of the periodic domain (null when one box covers it): the
  // domain cut into bins of own_bin cells per axis, bin b listing the boxes
  // own_box[own_start[b] .. own_start[b + 1]) that overlap it.
  const int* own_start;
  const int* own_box;
  int own_bin[3], own_dims[3];
};

struct Particles {
  const double* x;
  const double* y;
  const double* z;
  const double* a;  // CIC m, sinks a
  const double* b;  // SN m
  const double* c;  // SN e
  const double* r;  // SN r
  long long n;
  const long long* box_off;
};

// Tiles covering the padded (ghost-zoned) box of every box.  Along y and z,
// tile t covers padded cells [t*T, (t+1)*T) clipped to the padded extent.
// Along x the tile boundaries sit on owned cells, g + k*TX, so that a tile's
// owned x rows start on the state's cache-line boundaries: tile k covers
// [k == 0 ? 0 : g + k*TX, k == ntx-1 ? p : g + (k+1)*TX) with ntx =
// ceil(n/TX), so the first and last take the ghost slabs (width <= TX + 2g).
// Global tile id = tile_prefix[b] + (tz*nty + ty)*ntx + tx.
//
// Owner tiles (the fold-free step): tiles cover the owned cells only, [t*T,
// (t+1)*T) clipped to the box along every axis.  A particle is binned into
// every owner tile its stencil reaches after wrapping the stencil's cells
// periodically, in whichever box owns them, so a tile receives every
// contribution to its cells: what the ghost zones and the fold would carry is
// added where it lands.  Valid when no tile along an axis is wider than the
// domain less 2g cells: then a stencil (at most 2g + 1 cells per axis) meets
// at most one periodic image of a tile, and never holds two images of a cell.
// Geometry of one tile, fixed by the layout and the tile shape.
struct alignas(16) TileGeo {
  long long boff;  // buffer offset of the tile's box
  long long soff;  // state offset of the tile's box
  int p[3];        // padded extent of the box
  int o[3];        // tile origin, padded-local
  int ext[3];      // cells of the tile inside the padded box
  int b;           // box
  int glo[3];      // global cell of the tile origin (owner tiles: in [0, domain))
  int pad;
};

// Owner tiles: the box whose owned cells meet the region next to box b in
// direction (dx, dy, dz), d = 9 (dz + 1) + 3 (dy + 1) + (dx + 1) (per axis:
// the g cells below the box, the box's own extent, or the g cells above it,
// wrapped periodically), with what the binning needs of it: id -1 when no
// box does, -2 when several do (then the owner index is walked).
struct alignas(16) NbrBox {
  int id;
  int lo[3], n[3];
  int tprefix;  // its first owner tile
  int tax[3];   // its owner tiles per axis
  int pad;
};

struct TileGrid {
  int t[3];                       // tile edge per axis (TX, TY, TZ), powers of two
  int ts[3];                      // log2 t: a non-negative offset's tile is offset >> ts
  const long long* tile_prefix;   // [nbox+1] device
  const int* tiles_axis;          // [nbox][3] device: tiles per axis
  const TileGeo* geo;             // [ntiles] device
  long long ntiles;
  int gx;                         // ghost width (x tile boundaries at gx + k*TX)
  int wx;                         // widest x tile, TX + 2 gx (LDS row width)
  int owner;                      // 1: owner tiles (gx = 0, wx = TX)
  const NbrBox* nbr;              // owner tiles: [27 nbox] neighbour table
};

// A supernova as prepared once by the binning pass; tile entry lists hold
// particle indices into an array of these.
struct SnPk {
  double x, y, z, r;
  // share of each member cell: m / (N V) and e / (N V) as doubles, or, for
  // the fixed-point buffer, their 2^-40 quanta (int64 bits)
  double vr, ve;
  long long remr, reme;  // fixed point: Q(m / V) - N Q(m / (N V)), same for e
  int n;                 // sphere members (-1: host cell only, 0: skipped)
  int ti, tj, tk;        // padded-local remainder cell (owner tiles: its periodic image,
                         // global); ti < 0: none in the box
};

// A supernova entry of one tile as the tile pass holds it in LDS: the row
// test's inputs and the member share.
struct alignas(16) SnTile {
  double x, y, z, r2;     // centre and r^2
  double vr, ve;          // member share (for fixed point: the quanta's bits)
  int lo, hi;             // candidate cells along x, global (host cell alone: that cell)
  int host;               // bit 0: the host cell alone takes the deposit; owner tiles:
                          // bits 1 + 2a, 2 + 2a the tile image along axis a (+D, -D)
  unsigned rows;          // candidate tile rows: vlo | vhi << 8 | wlo << 16 | whi << 24
};

// Scratch for the binned deposit, owned by the context.  (particle, tile)
// pairs are bucket-sorted in two levels with LDS-only ranking: level 1 moves
// each pair's record into its coarse bucket (tile >> shift) through per-block
// histograms and a global scan; level 2 sorts each bucket by tile and writes
// the per-tile offsets.
struct BinWork {
  int shift;            // coarse bucket = tile >> shift
  int nbuckets;         // ceil(ntiles / 2^shift) <= 1024
  int nblk_cic, nblk_sn;  // level-1 blocks per kind
  int* hist;            // [nbuckets * (nblk_cic + nblk_sn) + 1]: histograms, then scanned
  int* block_sums;      // scan scratch
  double4* cic_tmp;     // level-1 output, grouped by bucket
  int* cic_tmp_tile;
  double4* cic_rec;     // level-2 output, grouped by tile
  int* cic_off;         // [ntiles + 1]
  int* sn_tmp;           // supernova entries: particle indices
  int* sn_tmp_tile;
  int* sn_rec;           // sorted by tile: particle index
  int* sn_off;          // [ntiles + 1]
  SnPk* sn_pk;          // [n_sn]
  long long cic_cap, sn_cap;
  // level 2 works on slices of at most kSlice records of one bucket
  int* slice_base;      // [2 * nbuckets + 1]: first slice of each (kind, bucket)
  int* hist2;           // [2^shift * max_slices + 1]: per (bucket, tile, slice), then scanned
  int* block_sums2;
  long long max_slices;
  // tiles with more entries than a chunk threshold are split over several
  // workgroups (chunk slots); each chunk leaves its LDS partial tile in
  // `partial` and the last one to finish combines them in chunk order
  int* heavy_base;      // [ntiles] first chunk slot of a split tile, or -1
  int* sink_flag;       // [ntiles] owner tiles with sinks: 1 where a sink kernel may reach
  int2* heavy_unit;     // [slot_cap] (tile, chunk) of each slot; tile -1: unused
  int* heavy_count;     // [1] chunk slots claimed this step (may exceed slot_cap)
  int* arrive;          // [slot_cap] finished chunks, at the tile's first slot
  void* partial;        // [slot_cap][2][lcells] 8-byte partial sums
  long long slot_cap;
};

constexpr int kSlice = 4096;

// Supernova entries per batch of the tile pass: one per lane of a wavefront.
constexpr int kTileSnBatch = 64;
// LDS of one tile workgroup: two accumulator channels of the widest tile
// (tx + 2g cells along x) with rows padded by one cell (and their two error
// bounds in the reproducibility mode), then one batch of supernova entries.
__host__ __device__ constexpr long long tile_lds_bytes_wx(int wx, int tyz, bool bounds) {
  return (bounds ? 4ll : 2ll) * (wx + 1) * tyz * tyz * 8 +
         (long long)kTileSnBatch * (long long)sizeof(SnTile);
}
__host__ __device__ constexpr long long tile_lds_bytes(int tx, int tyz, int g, bool bounds) {
  return tile_lds_bytes_wx(tx + 2 * g, tyz, bounds);
}

constexpr int kBinChunkCic = 1024;  // CIC particles per level-1 block
constexpr int kChunkBits = 10;      // log2 kBinChunkCic
static_assert(kBinChunkCic == 1 << kChunkBits, "chunk bits");
constexpr int kBinChunkSn = 256;    // supernovae per level-1 block (one per thread)

// Kernel launchers: all enqueue on `s` and return hipError_t of the launch.
hipError_t launch_zero(void* buf, long long bytes, int block, hipStream_t s);
hipError_t launch_cic_direct(const Mesh& M, const Particles& P, void* buf, int block,
                             hipStream_t s);
// Binned path: bin CIC and supernova particles into tiles, then one
// workgroup per tile accumulates in LDS and stores every field of its cells.
// cic or sn may be null.  Replaces the zero fill.  phase_bin/phase_tile
// bracket the two halves for the profiler.
hipError_t launch_bin(const Mesh& M, const TileGrid& T, const Particles* cic,
                      const Particles* sn, BinWork& bw, int count_lanes, hipStream_t s);
// Supernova tile records and the chunk table of split tiles (after launch_bin).
hipError_t launch_tile_prep(const Mesh& M, const TileGrid& T, const Particles* cic,
                            const Particles* sn, const BinWork& bw, const pmp_tuning& t,
                            hipStream_t s);
// state non-null: the step's Steps 3 + 5 are fused in for owned cells at
// least g from every face of their box (no ghost image reaches them); those
// cells' buffer entries are left unwritten, and launch_fold_apply finishes
// the shell cells.  With owner tiles (T.owner) every owned cell is applied
// and the buffer is not written, except in the tiles sink_flag marks (and
// with state null, in every tile), which are stored for the sink passes.
hipError_t launch_tile_deposit(const Mesh& M, const TileGrid& T, const Particles* cic,
                               const Particles* sn, const BinWork& bw, void* buf,
                               const pmp_tuning& t, void* state, const Limits& L,
                               hipStream_t s, const int* sink_flag = nullptr);
// Steps 2 + 3 + 5 for the shell cells only (after a fused tile pass).
hipError_t launch_fold_apply(const Mesh& M, void* state, const void* buf, const Limits& L,
                             hipStream_t s);
hipError_t launch_sn_direct(const Mesh& M, const Particles& P, void* buf, int lanes,
                            hipStream_t s);
// bound: the reproducibility mode's error bounds [buffer_elems] (else unused)
// Sink request parameters (pmp_sinks and the cell edge).  rate 1 is the
// Bondi-Hoyle rate and reads the sink mass and velocity arrays.
struct SinkParams {
  const double *m, *vx, *vy, *vz;
  double r_k, r_gauss, dx;
  double G, dt, gamma, lambda;
  int rate;
  int owner;  // the deposit adds to the owning box's cell (owner tiles: no fold follows)
};

// The sink scratch holds kSinkScratch doubles per sink: the kernel weight
// sum W, the requested mass and r_acc^2.
constexpr int kSinkScratch = 3;

// Owner tiles in a step with sinks: flags every owner tile a sink's kernel
// may reach (conservatively: its kernel cube widened by one cell), after
// clearing them all.
hipError_t launch_sink_tiles(const Mesh& M, const TileGrid& T, const Particles& sinks, double r_k,
                             int* flag, hipStream_t s);
// Steps 3 + 5 for the cells of the flagged owner tiles (the others were
// applied by the tile pass).
hipError_t launch_apply_tiles(const Mesh& M, const TileGrid& T, void* state, const void* buf,
                              const int* flag, const Limits& L, hipStream_t s);
hipError_t launch_sink_deposit(const Mesh& M, const Particles& P, const void* state,
                               void* buf, double* sink_scratch, const SinkParams& K,
                               const Limits& L, double* bound, hipStream_t s);
hipError_t launch_sink_update(const Mesh& M, const Particles& P, const void* state,
                              const void* buf, const double* sink_scratch, const SinkParams& K,
                              const Limits& L, double* dm, double* dpx, double* dpy,
                              double* dpz, hipStream_t s);
// Supernova remnants with the TIGRESS-variant deposit (pmp_snr).
struct SnrArgs {
  const double *x, *y, *z, *m, *e, *vx, *vy, *vz;
  long long n;
  const long long* box_off;
  double r_k, nh_per_rho, msf_coef, psnr_coef, eps_k;
  int sub;
};
hipError_t launch_snr_deposit(const Mesh& M, const SnrArgs& A, const void* state, void* buf,
                              double* info, hipStream_t s);

// Largest output list of one sink creation call (the index sort is
// quadratic in the number of new sinks).
constexpr long long kCreateMax = 65536;

// Existing sinks of a creation call: positions only (x, y, z device [n]).
struct SinkPos {
  const double *x, *y, *z;
  long long n;
};
hipError_t launch_sink_create(const Mesh& M, void* state, const void* buf, const SinkPos& E,
                              double r_k, const Limits& L, long long max_new, double* out,
                              long long* work, hipStream_t s);
hipError_t launch_fold(const Mesh& M, void* buf, int block, hipStream_t s);
hipError_t launch_apply(const Mesh& M, void* state, const void* buf, const Limits& L,
                        double* eta, int block, hipStream_t s);
hipError_t launch_clear_status(DevStatus* st, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, long long bytes, hipStream_t s);
// bytes a multiple of 64, 16-byte aligned
hipError_t launch_copy4(void* dst, const void* src, long long bytes, hipStream_t s);
hipError_t launch_atomic_bench(void* dst, long long slots, int type, int pattern,
                               long long n_ops, hipStream_t s);

}  // namespace pmp
