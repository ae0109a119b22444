// Internal device-side types and wavefront primitives of the docking library.
// gfx950 only: 64-lane wavefronts, DPP row operations, readlane.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "lg.h"

namespace lg {

// Grid as the kernels see it: the library stores the pocket with a one-node
// border of out_value on every side, so a clamp of the node index to [-1, n]
// replaces the per-axis range test of the nearest-voxel rule.  g0 points at
// padded node (1,1,1) = logical node (0,0,0); strides are the padded ones.
struct GridDev {
  const float* g0;
  const char* gb;   // padded grid, byte addressed: node (ix,iy,iz) in [-1,n]^3 sits at
  int bs[3];        //   gb + b0 + ix*bs[0] + iy*bs[1] + iz*bs[2] (bs = byte strides 4, 4(nx+2), ...)
  int b0;           //   b0 = byte offset of logical node (0,0,0); every offset is >= 0 and < 2^31
  // The scans read a second copy in 4x4x2-node bricks, one 128-byte cache line
  // each, so the samples of one lookup instruction (an arc or a short segment)
  // touch few lines.  Byte offset of padded node (px,py,pz) = Tx[px]+Ty[py]+Tz[pz]
  // with per-axis tables built in LDS by every block (brick_tables).
  const char* gk;
  int nb[3];        // bricks per axis
  int tab_base[3];  // first entry of each axis table in the LDS table array
  int tab_len;      // (nx+2)+(ny+2)+(nz+2) entries
  float c0[3];      // nearest-node map: f = fma(x, inv_h, c0), c0 = fma(-o, inv_h, 0.5)
  int n[3];
  int stride[3];    // 1, nx+2, (nx+2)(ny+2)
  float o[3];
  float fn[3];      // (float)n per axis
  float fn1[3];     // (float)(n-1) per axis, trilinear range
  float inv_h;
  float out;
};

struct LigDev {
  const int32_t* atom_offset;
  const int32_t* tors_offset;
  const float* x;
  const float* y;
  const float* z;
  const uint32_t* mask;
  const int32_t* tors_atoms;
  const float* inv_len;
  const float* ref;
};

struct DockDev {
  int R, A, T, S;
  float delta, clash2;
  float clash_r2;          // (sqrt(clash2) + margin)^2: pairs farther apart on their circles never clash
  int lazy_clash;          // 1: no pair list, test only the winner of each torsion scan
  float c[3];
  const float* restarts;   // [R][12]
  const float* angles;     // [A][2]
  float* final_scores;     // [n*R]
  uint16_t* moves;         // [R*S*(6n + total_torsions)]: selected sample of every scan;
                           // ligand i restart r sweep s at R*S*(6i + tors_offset[i]) + (r*S + s)*(6 + K_i)
  int16_t* trace;          // optional [n][R][S][trace_w]
  int trace_w;
};

// Refinement parameters and outputs.  kpl poses per ligand: pose i is member
// i % kpl of ligand i / kpl, its coordinates at kpl*atom_offset[lig] + member*N.
struct RefineDev {
  int steps, kpl;
  const int32_t* lig_ids;  // ligands of this launch (a size class), or nullptr: 0..n-1
  float eta_t, eta_w, eta_th, clip_t, clip_w, clip_th, clash2;
  float* xo;
  float* yo;
  float* zo;
  float* score;
};

// What differs between sites that share grid dimensions and spacing: the
// grid copies, the origin (and the nearest-node offsets built from it), the
// value outside the box and the site centre that placement moves ligands to.
// Sixteen 32-bit words, read into scalar registers.
struct SiteGrid {
  const float* g0;
  const char* gb;
  const char* gk;
  float c0[3];
  float o[3];
  float out;
  float c[3];
};

// Several docking sites in one launch: grids of identical dimensions and
// spacing (so one set of brick tables serves all); per site its own final
// scores and move records.  Items are (site, ligand, chunk), site by site or
// with the sites interleaved per ligand.
struct SitesDev {
  const SiteGrid* grids;    // device [n_sites]
  int n_sites;
  int site_major;           // 1: site by site; 0: every site of a ligand in turn
  size_t scores_stride;     // floats of final scores per site
  size_t moves_stride;      // move-record entries per site
};

// Persistent work source of one bucket: items are (ligand of the bucket,
// chunk of `chunk` restarts), pulled from `cursor` by whole wavefronts.
// LDS of a docking wavefront, in float4: scan data of 64*nslot atoms, two
// regions of 64*nslot float4 (risky torsion pairs or staged grid values), the
// ligand's fragment masks (one 32-bit word per atom).
constexpr int dock_wave_float4(int nslot) { return 3 * 64 * nslot + 16 * nslot; }

struct QueueDev {
  const int32_t* perm;          // ligand ids grouped by bucket
  const int32_t* bucket_start;  // [B+1]
  int32_t* cursor;              // one counter per bucket
  int bucket;
  int chunk;
};

// Cluster bounds of the device-side input preparation: atom cluster c holds
// ligands with atoms <= atom[c] (first match), rotamer cluster c bonds <= rot[c].
struct ClusterBounds {
  int na, nr;
  int atom[16];
  int rot[32];
};

// Radix-select state of the global ranking: the selected key prefix and its
// mask, how many keys of that prefix are still to take, whether the threshold is
// fixed, and the compaction counter.
struct RankState {
  uint64_t prefix, mask;
  uint32_t need, done, count, pad;
};

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Orders a wavefront's LDS writes before its later LDS reads by other lanes:
// waits for outstanding LDS operations and stops the compiler from moving
// memory operations across this point.
__device__ __forceinline__ void wave_sync() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

// Row-of-16 all-reduce with DPP, then the four row results through readlane.
// Needs all 64 lanes active.
template <class Op>
__device__ __forceinline__ int wave_reduce_i32(int v, Op op) {
  v = op(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true));   // quad_perm [1,0,3,2]
  v = op(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true));   // quad_perm [2,3,0,1]
  v = op(v, __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true));  // row_half_mirror
  v = op(v, __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true));  // row_mirror
  int a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
  int c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
  return op(op(a, b), op(c, d));
}

struct OpMax { __device__ int operator()(int a, int b) const { return a > b ? a : b; } };
struct OpMin { __device__ int operator()(int a, int b) const { return a < b ? a : b; } };
struct OpAddF {
  __device__ int operator()(int a, int b) const { return __float_as_int(__int_as_float(a) + __int_as_float(b)); }
};

__device__ __forceinline__ float wave_sum(float v) { return __int_as_float(wave_reduce_i32(__float_as_int(v), OpAddF())); }

// Per-axis byte-offset tables of the brick layout, indexed by padded node
// coordinate p in [0, n+1]: x (p>>2)*128 + (p&3)*4, y (p>>2)*128*nbx + (p&3)*16,
// z (p>>1)*128*nbx*nby + (p&1)*64.  Filled by all threads of a block.
__device__ __forceinline__ void fill_brick_tables(const GridDev& G, int* tab) {
  for (int k = threadIdx.x; k < G.tab_len; k += blockDim.x) {
    int a = k < G.tab_base[1] ? 0 : (k < G.tab_base[2] ? 1 : 2);
    int p = k - G.tab_base[a];
    int v;
    if (a == 0) v = (p >> 2) * 128 + (p & 3) * 4;
    else if (a == 1) v = (p >> 2) * 128 * G.nb[0] + (p & 3) * 16;
    else v = (p >> 1) * 128 * G.nb[0] * G.nb[1] + (p & 1) * 64;
    tab[k] = v;
  }
}

// 24-bit signed multiply-add (full-rate v_mad_i32_i24); |a| <= 1025, |b| < 2^23.
__device__ __forceinline__ int mad24(int a, int b, int c) { return __mul24(a, b) + c; }

// Grid value at a non-negative byte offset from the padded base (32-bit offset,
// scalar base address).
__device__ __forceinline__ float grid_at(const char* gb, int off) {
  return *reinterpret_cast<const float*>(gb + (uint32_t)off);
}

// Order-preserving map of a float to a signed int (total order on non-NaN).
__device__ __forceinline__ int orderable(float f) {
  int b = __float_as_int(f);
  return b ^ ((b >> 31) & 0x7FFFFFFF);
}

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

// Floor of f for a node map value already known to lie in [-1, n].
__device__ __forceinline__ int floor_node(float f) {
  int i;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(i) : "v"(f));
  return i;
}

// Node index on the padded grid for coordinate offset f (already scaled):
// floor of f clamped to [-1, n] -- -1 and n land on the out_value border.
__device__ __forceinline__ int clamp_node(float f, float fn) {
  f = __builtin_amdgcn_fmed3f(f, -1.0f, fn);
  int i;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(i) : "v"(f));
  return i;
}

}  // namespace lg
