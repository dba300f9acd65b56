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

// Device status word and counters (mirrors pmp_status).
struct DevStatus {
  unsigned int flags;
  unsigned int reserved;
  unsigned long long touched, bind, lam, fall;
};

struct Limits {
  double rho_floor, rho_tr, cap;
  int eint_mode;
};

// Everything a launch needs about the mesh.
struct Mesh {
  const DevBox* boxes;      // boxes this launch covers (all, or one for per-box launches)
  const DevBox* all_boxes;  // every box (fold sources)
  int nbox;
  int ghost;
  int domain[3];
  double V;
  int nfield;
  int acc;    // pmp_acc_t
  int state;  // pmp_state_t
  long long buffer_elems;
  long long owned_cells;
  const long long* owned_prefix;  // [nbox+1] cumulative owned cells
  const long long* shell_prefix;  // [nbox+1] cumulative shell cells
  const int* seg_off;             // [nbox+1] fold segments per destination box
  const DevSeg* segs;
  // Each box splits along every axis into [0, g), [g, n - g), [n - g, n) (27
  // zones); zone_off[28 b + z] .. zone_off[28 b + z + 1] index zone_seg, the
  // segments (in plan order) that reach zone z of box b.
  const int* zone_off;
  const int* zone_seg;
  // Work chunks of kChunk cells that never cross a box: (global box, first
  // cell) for the apply (owned cells) and for the fold (shell cells).
  const int2* apply_chunks;
  long long n_apply_chunks;
  const int2* fold_chunks;
  long long n_fold_chunks;
  long long shell_cells;
  DevStatus* status;
  int num_cu;
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

// Tiles covering the padded (ghost-zoned) box of every box: tile (tx,ty,tz)
// of box b covers padded local cells [tx*TX, (tx+1)*TX) x ... clipped to the
// padded extent.  Global tile id = tile_prefix[b] + (tz*nty + ty)*ntx + tx.
struct TileGrid {
  int t[3];                       // tile edge per axis (TX, TY, TZ)
  const long long* tile_prefix;   // [nbox+1] device
  const int* tiles_axis;          // [nbox][3] device: tiles per axis
  long long ntiles;
};

// A supernova as stored in its tiles' entry lists.
struct SnRec {
  double x, y, z, m, e, r;
  int n;       // sphere members (-1: host cell only)
  int target;  // padded-local index of the fixed-point remainder cell, or -1
};

// Scratch for the binned deposit, owned by the context.  The count pass
// records each (particle, tile) pair's slot in its tile, so the fill pass
// writes packed particle records without atomics.
struct BinWork {
  int* count;         // [2 * ntiles]: entries per tile, CIC tiles then supernova tiles
  int* offset;        // [2 * ntiles + 1]: exclusive scan of count
  int* block_sums;    // scan scratch [nblocks + 1]
  double4* cic_rec;   // [cic_cap] (x, y, z, m) grouped by tile
  SnRec* sn_rec;      // [sn_cap] grouped by tile
  int* cic_slot;      // [n_cic * 8] slot of each (particle, tile) pair
  int* sn_slot;       // [n_sn * sn_maxt]
  int* sn_n;          // [n_sn] members of each sphere (-1 host only, 0 skipped)
  int* sn_target;     // [n_sn]
  long long cic_cap, sn_cap;
  int sn_maxt;        // most tiles one supernova can touch
};

// Kernel launchers: all enqueue on `s` and return hipError_t of the launch.
hipError_t launch_zero(void* buf, long long bytes, int block, hipStream_t s);
hipError_t launch_cic_direct(const Mesh& M, const Particles& P, void* buf, int block,
                             hipStream_t s);
// Binned path: bin CIC and supernova particles into tiles, then one
// workgroup per tile accumulates in LDS and stores every field of its cells.
// cic or sn may be null.  Replaces the zero fill.  phase_bin/phase_tile
// bracket the two halves for the profiler.
hipError_t launch_bin(const Mesh& M, const TileGrid& T, const Particles* cic,
                      const Particles* sn, BinWork& bw, int block, hipStream_t s);
hipError_t launch_tile_deposit(const Mesh& M, const TileGrid& T, const Particles* cic,
                               const Particles* sn, const BinWork& bw, void* buf,
                               const pmp_tuning& t, hipStream_t s);
hipError_t launch_sn_direct(const Mesh& M, const Particles& P, void* buf, int lanes,
                            hipStream_t s);
hipError_t launch_sink_deposit(const Mesh& M, const Particles& P, const void* state,
                               void* buf, double* sink_scratch, double r_k, double r_gauss,
                               const Limits& L, hipStream_t s);
hipError_t launch_sink_update(const Mesh& M, const Particles& P, const void* state,
                              const void* buf, const double* sink_scratch, double r_k,
                              double r_gauss, const Limits& L, double* dm, double* dpx,
                              double* dpy, double* dpz, hipStream_t s);
hipError_t launch_fold(const Mesh& M, void* buf, int block, hipStream_t s);
// fold != 0: the ghost fold is done inside the apply (buffer left unfolded).
hipError_t launch_apply(const Mesh& M, void* state, const void* buf, const Limits& L,
                        double* eta, int block, int fold, hipStream_t s);
hipError_t launch_clear_status(DevStatus* st, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, long long bytes, hipStream_t s);

}  // namespace pmp
