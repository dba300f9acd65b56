// Internal declarations shared by the kernels (pmp_kernels.hip) and the host
// API (pmp_api.hip).  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pmp.h"

namespace pmp {

// One box of the layout, in device memory.
struct DevBox {
  int lo[3];        // first owned global cell
  int n[3];         // owned cells per axis
  int p[3];         // padded cells per axis (n + 2g)
  int pad_;
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
  const DevBox* boxes;
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

// Scratch for the binned deposit, owned by the context.
struct BinWork {
  int* key;           // [nparticles] tile id of each particle
  int* rank;          // [nparticles] arrival rank inside its tile
  int* perm;          // [nparticles] particles sorted by tile
  int* count;         // [ntiles + 1]
  int* offset;        // [ntiles + 1] exclusive scan of count
  int* block_sums;    // scan scratch
  int* chunk_count;   // [ntiles + 1] LDS work items per tile
  int* chunk_offset;  // [ntiles + 1] exclusive scan of chunk_count
  int* chunk_total;   // [1]
  const long long* tile_prefix;  // [nbox+1] cumulative tiles per box
  const int* tiles_per_axis;     // [nbox][3]
  long long ntiles;
  int scan_blocks;
};

// Kernel launchers: all enqueue on `s` and return hipError_t of the launch.
hipError_t launch_zero(void* buf, long long bytes, int block, hipStream_t s);
hipError_t launch_cic_direct(const Mesh& M, const Particles& P, void* buf, const BinWork* bw,
                             int dense_min, int block, hipStream_t s);
hipError_t launch_cic_binned(const Mesh& M, const Particles& P, void* buf, BinWork& bw,
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
hipError_t launch_apply(const Mesh& M, void* state, const void* buf, const Limits& L,
                        double* eta, int block, hipStream_t s);
hipError_t launch_clear_status(DevStatus* st, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, long long bytes, hipStream_t s);

}  // namespace pmp
