// Host side of the C ABI: validation, pocket handles, workspace, the plain
// per-ligand launch sequence, the bucketed persistent sequence captured as a
// HIP graph, scoring and ranking.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <thread>
#include <vector>

#include "host_checks.h"
#include "lg.h"
#include "lg_internal.h"

namespace lg {
hipError_t launch_dock_plain(int nslot, int spl, int wpb, const GridDev& G, const LigDev& Lg, const DockDev& D,
                             int lig, hipStream_t st);
hipError_t launch_dock_bucket(int nslot, int spl, int wpb, int blocks, const GridDev& G, const LigDev& Lg,
                              const DockDev& D, const QueueDev& Q, hipStream_t st);
hipError_t occupancy_dock_bucket(int nslot, int spl, int wpb, int tab_len, int* blocks_per_cu);
hipError_t launch_valu_probe(int kind, int blocks, int iters, float* out, hipStream_t st);
hipError_t launch_dock_sites(int nslot, int spl, int wpb, int blocks, const GridDev& G, const LigDev& Lg,
                             const DockDev& D, const QueueDev& Q, const SitesDev& Sd, hipStream_t st);
hipError_t attributes_dock_bucket(int nslot, int spl, hipFuncAttributes* attr);
hipError_t launch_topk(int nslot, const LigDev& Lg, const DockDev& D, int n, int k, float* score, int32_t* rid,
                       float* ox, float* oy, float* oz, float* all_scores, float* pivot, hipStream_t st);
hipError_t launch_score(const GridDev& G, const LigDev& P, int n, int interp, float* score, float* grad,
                        hipStream_t st);
size_t rank_scratch_bytes(int n, int m);
hipError_t launch_rank(const float* score, int n, int group, int m, void* work, int32_t* top_idx,
                       float* top_score, int32_t* top_member, hipStream_t st);
hipError_t rank_static_scratch(void** out, size_t* bytes);
hipError_t launch_pad(const float* src, int nx, int ny, int nz, float out, float* dst, hipStream_t st);
hipError_t launch_brick(const float* padded, int px, int py, int pz, int nbx, int nby, int nbz, float out,
                        float* brick, hipStream_t st);
hipError_t launch_bucketing(const int32_t* atom_offset, const int32_t* tors_offset, int n, const ClusterBounds& cb,
                            int32_t* cls, int32_t* counts, int32_t* start, int32_t* fill, int32_t* perm,
                            int32_t* cursors, hipStream_t st);
hipError_t launch_refine(int nslot, const GridDev& G, const LigDev& P, const RefineDev& Rp, int n, hipStream_t st);
hipError_t launch_refine_pair(const GridDev& G, const LigDev& P, const RefineDev& Rp, int n_lig, hipStream_t st);
hipError_t launch_score_moves(int nslot, const GridDev& G, const LigDev& P, const float* moves, int n, float* score,
                              float* grad, hipStream_t st);
hipError_t launch_check(const int32_t* atom_offset, const int32_t* tors_offset, const int32_t* tors_atoms, int n,
                        int total_atoms, int total_tors, int32_t* stats, hipStream_t st);
}  // namespace lg

namespace {

using lghost::fail;
using lghost::env_ll;
using lghost::workspace_limit;
using lghost::check_ligands;
using lghost::host_maxima;
using lghost::check_host_ligands;
using lghost::guarded;

#define LG_HIP(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return fail(LG_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Bump layout of a device workspace.
struct Layout {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  }
};

lg_tuning default_tuning() {
  lg_tuning t;
  std::memset(&t, 0, sizeof t);
  t.n_atom_clusters = 4;
  t.atom_bounds[0] = 64; t.atom_bounds[1] = 128; t.atom_bounds[2] = 192; t.atom_bounds[3] = 256;
  t.n_rot_clusters = 1;
  t.rot_bounds[0] = LG_MAX_TORSIONS;
  for (int i = 0; i < 4; ++i) t.waves_per_block[i] = 4;
  t.restart_chunk = 8;
  t.grid_scale = 1;
  t.plain_waves_per_block = 4;
  t.use_graph = 1;
  t.lazy_clash = 0;
  return t;
}

int spl_for(int A, int T) {
  int need = (std::max(A, T) + 63) / 64;
  int spl = 1;
  while (spl < need) spl *= 2;
  return spl;
}

}  // namespace

struct lg_pocket_s {
  int device = 0;
  int cus = 0;
  lg_pocket_desc desc{};
  float* padded = nullptr;
  float* brick = nullptr;
  lg::GridDev grid{};
  void* ws = nullptr;
  size_t ws_bytes = 0;
  lg_tuning tuning = default_tuning();
  hipGraphExec_t gexec = nullptr;
  std::vector<uint64_t> gkey;
  hipStream_t capture = nullptr;   // graphs are captured here, then launched on the caller's stream
  // per-bucket launches of the last call; timing events [0] before the first
  // launch, [1 + 2l] start and [2 + 2l] end of launch l, [1 + 2 nl] after the last
  std::vector<lg_bucket_stat> launches;
  std::vector<hipEvent_t> events;
  int32_t* counts_dev = nullptr;
  bool timed = false;
};

namespace {



lg_status ensure_ws(lg_pocket p, size_t bytes) {
  if (bytes <= p->ws_bytes) return LG_OK;
  const size_t limit = workspace_limit();
  if (bytes > limit)
    return fail(LG_ERR_OUT_OF_MEMORY, "workspace of %zu bytes exceeds LG_WORKSPACE_LIMIT = %zu", bytes, limit);
  if (p->gexec) {
    (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
    p->gkey.clear();
  }
  if (p->ws) {
    LG_HIP(hipDeviceSynchronize());
    LG_HIP(hipFree(p->ws));
    p->ws = nullptr;
    p->ws_bytes = 0;
  }
  size_t want = std::min(bytes + bytes / 8, limit);
  if (hipMalloc(&p->ws, want) != hipSuccess) {
    (void)hipGetLastError();
    p->ws = nullptr;
    return fail(LG_ERR_OUT_OF_MEMORY, "workspace of %zu bytes could not be allocated", want);
  }
  p->ws_bytes = want;
  return LG_OK;
}


// Device-side validation of offsets and bond ids (one small read-back).
lg_status check_on_device(lg_pocket p, const lg_ligands* L, int32_t* dstats, hipStream_t st, int* max_atoms,
                          int* max_tors) {
  int32_t h[6];
  LG_HIP(lg::launch_check(L->atom_offset, L->tors_offset, L->total_torsions > 0 ? L->tors_atoms : nullptr, L->n,
                          L->total_atoms, L->total_torsions, dstats, st));
  LG_HIP(hipMemcpyAsync(h, dstats, sizeof h, hipMemcpyDeviceToHost, st));
  LG_HIP(hipStreamSynchronize(st));
  (void)p;
  if (h[5] > 0) return fail(LG_ERR_INVALID_ARG, "%d ligands have offsets outside [0, total] or decreasing", h[5]);
  if (h[0] < 1 || h[1] > LG_MAX_ATOMS) return fail(LG_ERR_LIMIT, "atoms per ligand in [%d, %d], allowed 1..%d", h[0], h[1], LG_MAX_ATOMS);
  if (h[2] < 0 || h[3] > LG_MAX_TORSIONS) return fail(LG_ERR_LIMIT, "bonds per ligand in [%d, %d], allowed 0..%d", h[2], h[3], LG_MAX_TORSIONS);
  if (h[4] > 0) return fail(LG_ERR_INVALID_ARG, "%d rotatable bonds have atom ids out of range", h[4]);
  *max_atoms = h[1];
  *max_tors = h[3];
  return LG_OK;
}

lg::LigDev lig_dev(const lg_ligands* L) {
  lg::LigDev d;
  d.atom_offset = L->atom_offset;
  d.tors_offset = L->tors_offset;
  d.x = L->x;
  d.y = L->y;
  d.z = L->z;
  d.mask = L->frag_mask;
  d.tors_atoms = L->tors_atoms;
  d.inv_len = L->inv_bond_len;
  d.ref = L->ref_point;
  return d;
}

}  // namespace

extern "C" {


lg_status lg_load_pocket(const lg_pocket_desc* desc, const float* grid, int32_t grid_is_device, void* stream,
                         lg_pocket* out) {
  if (!desc || !grid || !out) return fail(LG_ERR_INVALID_ARG, "desc, grid and out must not be NULL");
  *out = nullptr;
  if (desc->nx < 2 || desc->ny < 2 || desc->nz < 2 || desc->nx > 1024 || desc->ny > 1024 || desc->nz > 1024)
    return fail(LG_ERR_LIMIT, "grid dims %d x %d x %d outside 2..1024", desc->nx, desc->ny, desc->nz);
  // byte offsets into the padded grid are 32-bit and plane strides 24-bit signed
  if (4LL * (desc->nx + 2) * (desc->ny + 2) >= (1LL << 23) ||
      128LL * ((desc->nx + 5) / 4) * ((desc->ny + 5) / 4) * ((desc->nz + 3) / 2) >= (1LL << 31))
    return fail(LG_ERR_LIMIT, "grid %d x %d x %d too large (padded plane < 2^21 nodes, volume < 2^29 nodes)",
                desc->nx, desc->ny, desc->nz);
  if (!(desc->spacing > 0.f) || !(desc->inv_spacing > 0.f) || !std::isfinite(desc->spacing))
    return fail(LG_ERR_INVALID_ARG, "spacing must be positive");
  int dev = 0;
  LG_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  LG_HIP(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(LG_ERR_UNSUPPORTED, "device %d is %s; this library is built for gfx950", dev, prop.gcnArchName);
  hipStream_t st = (hipStream_t)stream;
  lg_pocket p = new (std::nothrow) lg_pocket_s();
  if (!p) return fail(LG_ERR_OUT_OF_MEMORY, "host allocation failed");
  p->device = dev;
  p->cus = prop.multiProcessorCount;
  p->desc = *desc;
  const int nx = desc->nx, ny = desc->ny, nz = desc->nz;
  const size_t padded = (size_t)(nx + 2) * (ny + 2) * (nz + 2);
  if (hipMalloc(&p->padded, padded * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    delete p;
    return fail(LG_ERR_OUT_OF_MEMORY, "grid allocation failed");
  }
  lg_status s = LG_OK;
  if (grid_is_device) {
    if (lg::launch_pad(grid, nx, ny, nz, desc->out_value, p->padded, st) != hipSuccess)
      s = fail(LG_ERR_DEVICE, "pad kernel launch failed");
  } else {
    std::unique_ptr<float[]> h(new (std::nothrow) float[padded]);
    if (!h) {
      s = fail(LG_ERR_OUT_OF_MEMORY, "host copy of the padded grid (%zu bytes) could not be allocated",
               padded * sizeof(float));
    } else {
      std::fill(h.get(), h.get() + padded, desc->out_value);
      for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
          std::memcpy(&h[((size_t)(z + 1) * (ny + 2) + (y + 1)) * (nx + 2) + 1], &grid[((size_t)z * ny + y) * nx],
                      nx * sizeof(float));
      if (hipMemcpyAsync(p->padded, h.get(), padded * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        s = fail(LG_ERR_DEVICE, "grid upload failed");
    }
  }
  const int nbx = (nx + 2 + 3) / 4, nby = (ny + 2 + 3) / 4, nbz = (nz + 2 + 1) / 2;
  const size_t nbrick = (size_t)nbx * nby * nbz * 32;
  if (s == LG_OK && hipMalloc(&p->brick, nbrick * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    p->brick = nullptr;
    s = fail(LG_ERR_OUT_OF_MEMORY, "brick grid allocation failed");
  }
  if (s == LG_OK && lg::launch_brick(p->padded, nx + 2, ny + 2, nz + 2, nbx, nby, nbz, desc->out_value, p->brick, st) != hipSuccess)
    s = fail(LG_ERR_DEVICE, "brick kernel launch failed");
  if (s == LG_OK && hipStreamSynchronize(st) != hipSuccess) s = fail(LG_ERR_DEVICE, "stream synchronise failed");
  if (s != LG_OK) {
    (void)hipFree(p->padded);
    if (p->brick) (void)hipFree(p->brick);
    delete p;
    return s;
  }
  lg::GridDev& G = p->grid;
  G.stride[0] = 1;
  G.stride[1] = nx + 2;
  G.stride[2] = (nx + 2) * (ny + 2);
  G.g0 = p->padded + 1 + G.stride[1] + G.stride[2];
  G.gb = reinterpret_cast<const char*>(p->padded);
  for (int a = 0; a < 3; ++a) G.bs[a] = 4 * G.stride[a];
  G.b0 = 4 * (1 + G.stride[1] + G.stride[2]);
  G.n[0] = nx; G.n[1] = ny; G.n[2] = nz;
  for (int a = 0; a < 3; ++a) {
    G.o[a] = desc->origin[a];
    G.fn[a] = (float)G.n[a];
    G.fn1[a] = (float)(G.n[a] - 1);
  }
  G.inv_h = desc->inv_spacing;
  G.out = desc->out_value;
  for (int a = 0; a < 3; ++a) G.c0[a] = std::fma(-desc->origin[a], desc->inv_spacing, 0.5f);
  G.gk = reinterpret_cast<const char*>(p->brick);
  G.nb[0] = nbx; G.nb[1] = nby; G.nb[2] = nbz;
  G.tab_base[0] = 0;
  G.tab_base[1] = nx + 2;
  G.tab_base[2] = (nx + 2) + (ny + 2);
  G.tab_len = (nx + 2) + (ny + 2) + (nz + 2);
  if (hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking) != hipSuccess) {
    (void)hipFree(p->padded);
    (void)hipFree(p->brick);
    delete p;
    return fail(LG_ERR_DEVICE, "stream creation failed");
  }
  *out = p;
  return LG_OK;
}

lg_status lg_free_pocket(lg_pocket p) {
  if (!p) return LG_OK;
  (void)hipDeviceSynchronize();
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->capture) (void)hipStreamDestroy(p->capture);
  for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
  if (p->ws) (void)hipFree(p->ws);
  if (p->padded) (void)hipFree(p->padded);
  if (p->brick) (void)hipFree(p->brick);
  delete p;
  return LG_OK;
}

lg_status lg_set_tuning(lg_pocket p, const lg_tuning* t) {
  if (!p || !t) return fail(LG_ERR_INVALID_ARG, "pocket and tuning must not be NULL");
  lg_status s = lghost::check_tuning(t);
  if (s != LG_OK) return s;
  p->tuning = *t;
  if (p->gexec) {
    (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
    p->gkey.clear();
  }
  return LG_OK;
}

lg_status lg_get_tuning(lg_pocket p, lg_tuning* t) {
  if (!p || !t) return fail(LG_ERR_INVALID_ARG, "pocket and tuning must not be NULL");
  *t = p->tuning;
  return LG_OK;
}

}  // extern "C"

// Workspace of one docking call: validation counters, final scores, move
// records, bucket arrays.
struct DockWs {
  size_t stats, final_scores, moves, cls, perm, cnt, bytes;
};

DockWs dock_ws_layout(int n, int R, int S, long long total_torsions, int buckets) {
  Layout lay;
  DockWs w;
  w.stats = lay.take(16 * sizeof(int32_t));
  w.final_scores = lay.take((size_t)n * R * sizeof(float));
  w.moves = lay.take((size_t)R * S * (6 * (size_t)n + (size_t)total_torsions) * sizeof(uint16_t));
  w.cls = lay.take((size_t)n * sizeof(int32_t));
  w.perm = lay.take((size_t)n * sizeof(int32_t));
  w.cnt = lay.take((size_t)(4 * buckets + 1) * sizeof(int32_t));
  w.bytes = lay.off;
  return w;
}

// Docking of one batch.  host_max_atoms >= 0: the batch was validated on the
// host (largest ligand and bond count given), no device check and read-back;
// direct: launch on the stream even when the tuning asks for a graph.
lg_status dock_batch_impl(lg_pocket p, const lg_ligands* L, const lg_dock_params* P, const lg_dock_out* O,
                          void* stream, int host_max_atoms, int host_max_tors, bool direct) {
  if (!p || !P || !O) return fail(LG_ERR_INVALID_ARG, "pocket, params and out must not be NULL");
  lg_status s = check_ligands(L, true);
  if (s != LG_OK) return s;
  if (P->restarts < 1 || P->restarts > LG_MAX_RESTARTS) return fail(LG_ERR_LIMIT, "restarts %d outside 1..%d", P->restarts, LG_MAX_RESTARTS);
  if (P->angle_samples < 1 || P->angle_samples > LG_MAX_SAMPLES || P->trans_samples < 1 || P->trans_samples > LG_MAX_SAMPLES)
    return fail(LG_ERR_LIMIT, "samples per scan outside 1..%d", LG_MAX_SAMPLES);
  if (P->sweeps < 0) return fail(LG_ERR_INVALID_ARG, "sweeps < 0");
  if (P->top_k < 1 || P->top_k > P->restarts) return fail(LG_ERR_INVALID_ARG, "top_k %d outside 1..R", P->top_k);
  if (P->mode != LG_PLAIN && P->mode != LG_BUCKETED) return fail(LG_ERR_INVALID_ARG, "unknown mode %d", P->mode);
  if (!P->restart_table || !P->angle_table) return fail(LG_ERR_INVALID_ARG, "restart_table and angle_table are required");
  if (!std::isfinite(P->trans_step) || !std::isfinite(P->clash_dist2)) return fail(LG_ERR_INVALID_ARG, "non-finite step or clash distance");
  if (L->n > 0 && (!O->score || !O->restart_id || !O->x || !O->y || !O->z))
    return fail(LG_ERR_INVALID_ARG, "score, restart_id and x/y/z outputs are required");
  if (L->n == 0) return LG_OK;
  if ((long long)P->restarts * P->sweeps * (6LL * L->n + L->total_torsions) > (1LL << 40))
    return fail(LG_ERR_LIMIT, "R * sweeps * (6 n + total_torsions) move records too large");
  // the persistent launches take work items (ligand, restart chunk) from a 32-bit
  // cursor that every wavefront advances once past the end
  const lg_tuning& tu = p->tuning;
  if (P->mode == LG_BUCKETED &&
      (long long)L->n * ((P->restarts + tu.restart_chunk - 1) / tu.restart_chunk) >= (1LL << 30))
    return fail(LG_ERR_LIMIT, "ligands x restart chunks (%d x %d) must stay below 2^30 work items", L->n,
                (P->restarts + tu.restart_chunk - 1) / tu.restart_chunk);
  hipStream_t st = (hipStream_t)stream;
  LG_HIP(hipSetDevice(p->device));

  const int n = L->n, R = P->restarts;
  const int B = tu.n_atom_clusters * tu.n_rot_clusters;
  const DockWs wl = dock_ws_layout(n, R, P->sweeps, L->total_torsions, B);
  const size_t o_final = wl.final_scores, o_moves = wl.moves, o_cls = wl.cls, o_perm = wl.perm, o_cnt = wl.cnt;
  s = ensure_ws(p, wl.bytes);
  if (s != LG_OK) return s;
  char* ws = (char*)p->ws;
  int32_t* stats = (int32_t*)(ws + wl.stats);

  int max_atoms = host_max_atoms, max_tors = host_max_tors;
  if (max_atoms < 0) host_maxima(L, &max_atoms, &max_tors);
  if (max_atoms < 0) {
    s = check_on_device(p, L, stats, st, &max_atoms, &max_tors);
    if (s != LG_OK) return s;
  }
  if (O->trace && O->trace_kmax < max_tors) return fail(LG_ERR_INVALID_ARG, "trace_kmax %d < largest bond count %d", O->trace_kmax, max_tors);

  lg::DockDev D;
  D.R = R;
  D.A = P->angle_samples;
  D.T = P->trans_samples;
  D.S = P->sweeps;
  D.delta = P->trans_step;
  D.clash2 = P->clash_dist2;
  // 0.05 A margin of the risky-pair bound (the FP32 rotation stays within ~1e-5 A of the circle)
  D.clash_r2 = P->clash_dist2 > 0.f ? (std::sqrt(P->clash_dist2) + 0.05f) * (std::sqrt(P->clash_dist2) + 0.05f) : 0.f;
  for (int a = 0; a < 3; ++a) D.c[a] = p->desc.center[a];
  D.restarts = P->restart_table;
  D.angles = P->angle_table;
  D.final_scores = (float*)(ws + o_final);
  D.moves = (uint16_t*)(ws + o_moves);
  D.lazy_clash = tu.lazy_clash;
  D.trace = O->trace;
  D.trace_w = 6 + (O->trace ? O->trace_kmax : 0);
  const lg::LigDev Lg = lig_dev(L);
  const int topk_slots = std::max(1, (max_atoms + 63) / 64);   // replay instance for the largest ligand
  const int spl = spl_for(D.A, D.T);
  if (spl > 16) return fail(LG_ERR_LIMIT, "samples per lane %d > 16", spl);

  if (P->mode == LG_PLAIN) {
    // the plain method: one launch per ligand, kernel sized for the largest class
    const int nslot = LG_MAX_ATOMS / 64;
    for (int i = 0; i < n; ++i)
      LG_HIP(lg::launch_dock_plain(nslot, spl, tu.plain_waves_per_block, p->grid, Lg, D, i, st));
    LG_HIP(lg::launch_topk(topk_slots, Lg, D, n, P->top_k, O->score, O->restart_id, O->x, O->y, O->z, O->all_scores,
                           O->pivot, st));
    return LG_OK;
  }

  // bucketed: classify / scan / scatter on the device, one persistent launch per
  // bucket, top-k; captured once as a graph and replayed for identical calls
  int32_t* cls = (int32_t*)(ws + o_cls);
  int32_t* perm = (int32_t*)(ws + o_perm);
  int32_t* counts = (int32_t*)(ws + o_cnt);
  int32_t* start = counts + B;
  int32_t* fill = start + B + 1;
  int32_t* cursors = fill + B;
  std::vector<uint64_t> key = {(uint64_t)n, (uint64_t)L->total_atoms,
                               (uint64_t)L->total_torsions, (uint64_t)(uintptr_t)p->ws,
                               (uint64_t)R, (uint64_t)D.A, (uint64_t)D.T, (uint64_t)D.S, (uint64_t)P->top_k};
  const void* ptrs[] = {L->atom_offset, L->tors_offset, L->x, L->y, L->z, L->frag_mask, L->tors_atoms,
                        L->inv_bond_len, L->ref_point, P->restart_table, P->angle_table, O->score,
                        O->restart_id, O->x, O->y, O->z, O->all_scores, O->trace, O->pivot};
  for (const void* q : ptrs) key.push_back((uint64_t)(uintptr_t)q);
  uint32_t fb[3];
  std::memcpy(&fb[0], &D.delta, 4);
  std::memcpy(&fb[1], &D.clash2, 4);
  fb[2] = (uint32_t)O->trace_kmax;
  for (uint32_t v : fb) key.push_back(v);
  key.push_back((uint64_t)max_atoms);   // sizes the kernel instances of the plan

  lg::ClusterBounds cb;
  std::memset(&cb, 0, sizeof cb);
  cb.na = tu.n_atom_clusters;
  cb.nr = tu.n_rot_clusters;
  for (int c = 0; c < cb.na; ++c) cb.atom[c] = tu.atom_bounds[c];
  for (int c = 0; c < cb.nr; ++c) cb.rot[c] = tu.rot_bounds[c];
  // every atom cluster must fit its kernel instance: the last one takes the rest
  cb.atom[cb.na - 1] = LG_MAX_ATOMS;

  auto plan = [&](std::vector<lg_bucket_stat>& launches) -> lg_status {
    // Eq. 1: resident blocks per CU of each instance give the persistent grid
    for (int ca = cb.na - 1; ca >= 0; --ca) {
      // the instance holds the cluster's largest possible ligand: its bound, or the
      // batch's largest ligand if that is smaller (the last bound is LG_MAX_ATOMS)
      const int nslot = std::max(1, (std::min(cb.atom[ca], max_atoms) + 63) / 64);
      const int wpb = tu.waves_per_block[nslot - 1];
      int bpc = 0;
      LG_HIP(lg::occupancy_dock_bucket(nslot, spl, wpb, p->grid.tab_len, &bpc));
      if (bpc < 1) return fail(LG_ERR_DEVICE, "kernel instance (%d slots, %d samples/lane) cannot be resident", nslot, spl);
      hipFuncAttributes attr;
      LG_HIP(lg::attributes_dock_bucket(nslot, spl, &attr));
      for (int cr = cb.nr - 1; cr >= 0; --cr) {
        lg_bucket_stat b;
        b.bucket = ca * cb.nr + cr;
        b.atom_bound = cb.atom[ca];
        b.rot_bound = cb.rot[cr];
        b.slots = nslot;
        b.samples_per_lane = spl;
        b.waves_per_block = wpb;
        b.vgprs = attr.numRegs;
        b.lds_bytes = (int32_t)((size_t)((p->grid.tab_len + 3) & ~3) * 4 + (size_t)wpb * lg::dock_wave_float4(nslot) * 16);
        b.blocks_per_cu = bpc;
        b.blocks = bpc * p->cus * tu.grid_scale;
        b.ligands = -1;
        b.ms = -1.f;
        launches.push_back(b);
      }
    }
    const size_t nl = launches.size();
    p->events.reserve(2 * nl + 2);   // a failed allocation throws here, before an event exists
    while (p->events.size() < 2 * nl + 2) {
      hipEvent_t ev;
      LG_HIP(hipEventCreate(&ev));
      p->events.push_back(ev);
    }
    return LG_OK;
  };
  // The whole bucketed sequence on stream `cs`: bucketing, the bucket launches
  // one after another, largest instance first, then the top-k.  `timed`: events
  // around every launch.  (Launches on separate streams were tried: they overlap
  // when launched directly but were slower than this sequence, and graph replays
  // ran them one after another anyway.)
  auto enqueue = [&](const std::vector<lg_bucket_stat>& launches, hipStream_t cs, bool timed) -> hipError_t {
    const size_t nl = launches.size();
    hipError_t e = lg::launch_bucketing(L->atom_offset, L->tors_offset, n, cb, cls, counts, start, fill, perm, cursors, cs);
    if (e == hipSuccess && timed) e = hipEventRecord(p->events[0], cs);
    for (size_t l = 0; l < nl && e == hipSuccess; ++l) {
      const lg_bucket_stat& b = launches[l];
      if (timed) e = hipEventRecord(p->events[1 + 2 * l], cs);
      lg::QueueDev Q{perm, start, cursors, b.bucket, tu.restart_chunk};
      if (e == hipSuccess) e = lg::launch_dock_bucket(b.slots, spl, b.waves_per_block, b.blocks, p->grid, Lg, D, Q, cs);
      if (e == hipSuccess && timed) e = hipEventRecord(p->events[2 + 2 * l], cs);
    }
    if (e == hipSuccess && timed) e = hipEventRecord(p->events[1 + 2 * nl], cs);
    if (e == hipSuccess)
      e = lg::launch_topk(topk_slots, Lg, D, n, P->top_k, O->score, O->restart_id, O->x, O->y, O->z, O->all_scores,
                          O->pivot, cs);
    return e;
  };

  if (!tu.use_graph || direct) {
    std::vector<lg_bucket_stat> launches;
    s = plan(launches);
    if (s != LG_OK) return s;
    hipError_t e = enqueue(launches, st, true);
    if (e != hipSuccess) return fail(LG_ERR_DEVICE, "bucketed launch failed: %s", hipGetErrorString(e));
    p->launches = std::move(launches);
    p->counts_dev = counts;
    p->timed = true;
    return LG_OK;
  }
  if (!p->gexec || key != p->gkey) {
    if (p->gexec) {
      (void)hipGraphExecDestroy(p->gexec);
      p->gexec = nullptr;
      p->gkey.clear();
    }
    std::vector<lg_bucket_stat> launches;
    s = plan(launches);
    if (s != LG_OK) return s;
    hipGraph_t graph = nullptr;
    hipStream_t cs = p->capture;
    LG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
    hipError_t e = enqueue(launches, cs, false);
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return fail(LG_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipError_t e3 = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) {
      p->gexec = nullptr;
      return fail(LG_ERR_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e3));
    }
    p->gkey = std::move(key);
    p->launches = std::move(launches);
    p->counts_dev = counts;
  }
  p->timed = false;
  LG_HIP(hipGraphLaunch(p->gexec, st));
  return LG_OK;
}


extern "C" {

lg_status lg_dock_batch(lg_pocket p, const lg_ligands* L, const lg_dock_params* P, const lg_dock_out* O,
                        void* stream) {
  return guarded([&] { return dock_batch_impl(p, L, P, O, stream, -1, -1, false); });
}

}  // extern "C"

namespace {

lg_status dock_stream_impl(lg_pocket p, const lg_host_ligands* H, const lg_dock_params* P, int32_t chunk,
                           const lg_host_out* O, void* stream) {
  if (!p || !P || !O) return fail(LG_ERR_INVALID_ARG, "pocket, params and out must not be NULL");
  lg_status s = check_host_ligands(H);
  if (s != LG_OK) return s;
  if (chunk < 1) return fail(LG_ERR_INVALID_ARG, "chunk %d < 1", chunk);
  if (P->top_k < 1 || P->top_k > P->restarts || P->restarts > LG_MAX_RESTARTS)
    return fail(LG_ERR_INVALID_ARG, "top_k %d outside 1..R", P->top_k);
  if (H->n > 0 && (!O->score || !O->restart_id || !O->x || !O->y || !O->z))
    return fail(LG_ERR_INVALID_ARG, "score, restart_id and x/y/z outputs are required");
  if (H->n == 0) return LG_OK;
  const int k = P->top_k;
  hipStream_t cs = (hipStream_t)stream;
  LG_HIP(hipSetDevice(p->device));

  // chunks of consecutive ligands; per chunk its largest ligand and bond count
  struct Chunk { int c0, c1, max_atoms, max_tors; };
  std::vector<Chunk> chunks;
  int cap_n = 0, cap_atoms = 0, cap_tors = 0, mx_tors = 0;
  for (int c0 = 0; c0 < H->n; c0 += chunk) {
    Chunk c{c0, std::min(H->n, c0 + chunk), 0, 0};
    for (int i = c.c0; i < c.c1; ++i) {
      c.max_atoms = std::max(c.max_atoms, H->atom_offset[i + 1] - H->atom_offset[i]);
      c.max_tors = std::max(c.max_tors, H->tors_offset[i + 1] - H->tors_offset[i]);
    }
    cap_n = std::max(cap_n, c.c1 - c.c0);
    cap_atoms = std::max(cap_atoms, H->atom_offset[c.c1] - H->atom_offset[c.c0]);
    cap_tors = std::max(cap_tors, H->tors_offset[c.c1] - H->tors_offset[c.c0]);
    mx_tors = std::max(mx_tors, c.max_tors);
    chunks.push_back(c);
  }
  // the chunks still to dock (a resume manifest marks finished ones)
  std::vector<int> todo;
  for (int ci = 0; ci < (int)chunks.size(); ++ci)
    if (!O->chunk_done || O->chunk_done[ci] == 0) todo.push_back(ci);
  if (todo.empty()) return LG_OK;
  // the workspace of the largest chunk, allocated before anything is in flight
  s = ensure_ws(p, dock_ws_layout(cap_n, P->restarts, P->sweeps, cap_tors,
                                  p->tuning.n_atom_clusters * p->tuning.n_rot_clusters).bytes);
  if (s != LG_OK) return s;

  // one slot = device inputs + outputs of a chunk and their pinned host staging
  Layout lay;
  const size_t o_aoff = lay.take((size_t)(cap_n + 1) * 4), o_toff = lay.take((size_t)(cap_n + 1) * 4);
  const size_t o_x = lay.take((size_t)cap_atoms * 4), o_y = lay.take((size_t)cap_atoms * 4);
  const size_t o_z = lay.take((size_t)cap_atoms * 4), o_mask = lay.take((size_t)cap_atoms * 4);
  const size_t o_tat = lay.take((size_t)2 * cap_tors * 4 + 4), o_il = lay.take((size_t)cap_tors * 4 + 4);
  const size_t o_ref = lay.take((size_t)3 * cap_n * 4);
  const size_t o_sc = lay.take((size_t)cap_n * k * 4), o_rid = lay.take((size_t)cap_n * k * 4);
  const size_t o_piv = lay.take((size_t)3 * cap_n * k * 4);
  const size_t o_ox = lay.take((size_t)k * cap_atoms * 4), o_oy = lay.take((size_t)k * cap_atoms * 4);
  const size_t o_oz = lay.take((size_t)k * cap_atoms * 4);
  const size_t slot_bytes = lay.off;
  char* dev[2] = {nullptr, nullptr};
  char* host[2] = {nullptr, nullptr};
  hipStream_t cin = nullptr, cout = nullptr;
  hipEvent_t ev_in[2] = {}, ev_dock[2] = {}, ev_out[2] = {};
  auto release = [&]() {
    (void)hipStreamSynchronize(cs);
    for (int i = 0; i < 2; ++i) {
      if (ev_out[i]) (void)hipEventSynchronize(ev_out[i]);
    }
    if (cin) (void)hipStreamSynchronize(cin);
    if (cout) (void)hipStreamSynchronize(cout);
    for (int i = 0; i < 2; ++i) {
      if (dev[i]) (void)hipFree(dev[i]);
      if (host[i]) (void)hipHostFree(host[i]);
      for (hipEvent_t e : {ev_in[i], ev_dock[i], ev_out[i]})
        if (e) (void)hipEventDestroy(e);
    }
    if (cin) (void)hipStreamDestroy(cin);
    if (cout) (void)hipStreamDestroy(cout);
  };
  if (2 * slot_bytes > workspace_limit())
    return fail(LG_ERR_OUT_OF_MEMORY, "stream buffers of 2 x %zu bytes exceed LG_WORKSPACE_LIMIT = %zu", slot_bytes,
                workspace_limit());
  bool ok = true;
  for (int i = 0; i < 2 && ok; ++i) {
    ok = hipMalloc((void**)&dev[i], slot_bytes) == hipSuccess &&
         hipHostMalloc((void**)&host[i], slot_bytes, hipHostMallocDefault) == hipSuccess &&
         hipEventCreateWithFlags(&ev_in[i], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&ev_dock[i], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&ev_out[i], hipEventDisableTiming) == hipSuccess;
  }
  ok = ok && hipStreamCreateWithFlags(&cin, hipStreamNonBlocking) == hipSuccess &&
       hipStreamCreateWithFlags(&cout, hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    release();
    return fail(LG_ERR_OUT_OF_MEMORY, "stream buffers (2 x %zu bytes device and pinned host) could not be allocated", slot_bytes);
  }

  // results of the chunk at position t of todo (slot t % 2, copied back) into
  // the caller's arrays, then its manifest entry
  auto unpack = [&](int t) {
    const Chunk& c = chunks[todo[t]];
    const char* h = host[t % 2];
    const size_t nk = (size_t)(c.c1 - c.c0) * k;
    const size_t a0 = (size_t)H->atom_offset[c.c0], na = (size_t)H->atom_offset[c.c1] - a0;
    // the pose coordinates (most of the bytes, often into pages the caller has
    // not touched yet) in page-aligned slices of at least 1 MB per array, one
    // thread per slice beyond the first (up to eight slices); a slice whose
    // thread cannot start is copied here
    const size_t pose_bytes = (size_t)k * na * 4;
    char* dst[3] = {(char*)(O->x + k * a0), (char*)(O->y + k * a0), (char*)(O->z + k * a0)};
    const char* src[3] = {h + o_ox, h + o_oy, h + o_oz};
    constexpr int kMaxSlices = 8;
    const int slices = (int)std::max<size_t>(1, std::min<size_t>(kMaxSlices, pose_bytes >> 20));
    auto slice = [&](int s) {
      size_t b0, b1;
      lghost::copy_slice(pose_bytes, slices, s, &b0, &b1);
      if (b1 > b0)
        for (int d = 0; d < 3; ++d) std::memcpy(dst[d] + b0, src[d] + b0, b1 - b0);
    };
    std::thread th[kMaxSlices - 1];
    for (int s = 1; s < slices; ++s) {
      try {
        th[s - 1] = std::thread(slice, s);
      } catch (...) {
        slice(s);
      }
    }
    slice(0);
    std::memcpy(O->score + (size_t)c.c0 * k, h + o_sc, nk * 4);
    std::memcpy(O->restart_id + (size_t)c.c0 * k, h + o_rid, nk * 4);
    if (O->pivot) std::memcpy(O->pivot + (size_t)c.c0 * k * 3, h + o_piv, nk * 12);
    for (std::thread& w : th)
      if (w.joinable()) w.join();
    if (O->chunk_done) {
      std::atomic_thread_fence(std::memory_order_release);   // outputs before the entry
      reinterpret_cast<volatile int32_t*>(O->chunk_done)[todo[t]] = 1;
    }
  };
  auto copy = [&](void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t st) -> hipError_t {
    return bytes ? hipMemcpyAsync(dst, src, bytes, kind, st) : hipSuccess;
  };

  const int nc = (int)todo.size();
  const long long fault_after = env_ll("LG_FAULT_AFTER_CHUNKS", -1);
  int enq = 0;   // chunks of todo enqueued (docking and copy-back)
  for (int ci = 0; ci < nc && s == LG_OK; ++ci) {
    if (ci == fault_after) break;
    const Chunk& c = chunks[todo[ci]];
    const int sl = ci % 2;
    char* h = host[sl];
    char* d = dev[sl];
    // the slot's previous chunk (ci - 2) was unpacked after chunk ci - 1 was
    // enqueued, so its staging is free
    // pack: offsets rebased to the chunk, arrays copied into pinned staging
    const int n = c.c1 - c.c0;
    const int a0 = H->atom_offset[c.c0], na = H->atom_offset[c.c1] - a0;
    const int t0 = H->tors_offset[c.c0], nt = H->tors_offset[c.c1] - t0;
    int32_t* ao = (int32_t*)(h + o_aoff);
    int32_t* to = (int32_t*)(h + o_toff);
    for (int i = 0; i <= n; ++i) {
      ao[i] = H->atom_offset[c.c0 + i] - a0;
      to[i] = H->tors_offset[c.c0 + i] - t0;
    }
    std::memcpy(h + o_x, H->x + a0, (size_t)na * 4);
    std::memcpy(h + o_y, H->y + a0, (size_t)na * 4);
    std::memcpy(h + o_z, H->z + a0, (size_t)na * 4);
    std::memcpy(h + o_mask, H->frag_mask + a0, (size_t)na * 4);
    if (nt > 0) {
      std::memcpy(h + o_tat, H->tors_atoms + 2 * (size_t)t0, (size_t)nt * 8);
      std::memcpy(h + o_il, H->inv_bond_len + t0, (size_t)nt * 4);
    }
    std::memcpy(h + o_ref, H->ref_point + 3 * (size_t)c.c0, (size_t)n * 12);
    // copy in once the slot's previous docking no longer reads its inputs
    hipError_t e = hipSuccess;
    if (ci >= 2) e = hipStreamWaitEvent(cin, ev_dock[sl], 0);
    for (size_t off : {o_aoff, o_toff})
      if (e == hipSuccess) e = copy(d + off, h + off, (size_t)(n + 1) * 4, hipMemcpyHostToDevice, cin);
    for (size_t off : {o_x, o_y, o_z, o_mask})
      if (e == hipSuccess) e = copy(d + off, h + off, (size_t)na * 4, hipMemcpyHostToDevice, cin);
    if (e == hipSuccess) e = copy(d + o_tat, h + o_tat, (size_t)nt * 8, hipMemcpyHostToDevice, cin);
    if (e == hipSuccess) e = copy(d + o_il, h + o_il, (size_t)nt * 4, hipMemcpyHostToDevice, cin);
    if (e == hipSuccess) e = copy(d + o_ref, h + o_ref, (size_t)n * 12, hipMemcpyHostToDevice, cin);
    if (e == hipSuccess) e = hipEventRecord(ev_in[sl], cin);
    if (e == hipSuccess) e = hipStreamWaitEvent(cs, ev_in[sl], 0);
    if (e != hipSuccess) { s = fail(LG_ERR_DEVICE, "stream copy-in failed: %s", hipGetErrorString(e)); break; }
    // dock the chunk on the caller's stream
    lg_ligands L;
    L.n = n;
    L.total_atoms = na;
    L.total_torsions = nt;
    L.atom_offset = (const int32_t*)(d + o_aoff);
    L.tors_offset = (const int32_t*)(d + o_toff);
    L.x = (const float*)(d + o_x);
    L.y = (const float*)(d + o_y);
    L.z = (const float*)(d + o_z);
    L.frag_mask = (const uint32_t*)(d + o_mask);
    L.tors_atoms = (const int32_t*)(d + o_tat);
    L.inv_bond_len = (const float*)(d + o_il);
    L.ref_point = (const float*)(d + o_ref);
    L.atom_offset_host = ao;
    L.tors_offset_host = to;
    L.tors_atoms_host = nullptr;   // checked with the library; maxima passed below
    lg_dock_out DO;
    std::memset(&DO, 0, sizeof DO);
    DO.score = (float*)(d + o_sc);
    DO.restart_id = (int32_t*)(d + o_rid);
    DO.pivot = (float*)(d + o_piv);
    DO.x = (float*)(d + o_ox);
    DO.y = (float*)(d + o_oy);
    DO.z = (float*)(d + o_oz);
    lg_dock_params DP = *P;
    DP.mode = LG_BUCKETED;
    s = guarded([&] { return dock_batch_impl(p, &L, &DP, &DO, cs, c.max_atoms, c.max_tors, true); });
    if (s != LG_OK) break;
    e = hipEventRecord(ev_dock[sl], cs);
    // copy the results out behind the docking
    if (e == hipSuccess) e = hipStreamWaitEvent(cout, ev_dock[sl], 0);
    const size_t nk = (size_t)n * k;
    for (size_t off : {o_sc, o_rid})
      if (e == hipSuccess) e = copy(h + off, d + off, nk * 4, hipMemcpyDeviceToHost, cout);
    if (e == hipSuccess && O->pivot) e = copy(h + o_piv, d + o_piv, nk * 12, hipMemcpyDeviceToHost, cout);
    for (size_t off : {o_ox, o_oy, o_oz})
      if (e == hipSuccess) e = copy(h + off, d + off, (size_t)k * na * 4, hipMemcpyDeviceToHost, cout);
    if (e == hipSuccess) e = hipEventRecord(ev_out[sl], cout);
    if (e != hipSuccess) { s = fail(LG_ERR_DEVICE, "stream copy-out failed: %s", hipGetErrorString(e)); break; }
    enq = ci + 1;
    // the previous chunk's results into the caller's arrays while this one docks
    if (ci >= 1) {
      if (hipEventSynchronize(ev_out[(ci - 1) % 2]) != hipSuccess) {
        s = fail(LG_ERR_DEVICE, "stream copy-back failed");
        break;
      }
      unpack(ci - 1);
    }
  }
  // the last chunk enqueued
  if (s == LG_OK && enq >= 1) {
    if (hipEventSynchronize(ev_out[(enq - 1) % 2]) != hipSuccess)
      s = fail(LG_ERR_DEVICE, "stream copy-back failed");
    else
      unpack(enq - 1);
  }
  release();
  if (s == LG_OK && enq < nc)
    s = fail(LG_ERR_DEVICE, "stopped after %d of %d chunks (LG_FAULT_AFTER_CHUNKS)", enq, nc);
  return s;
}

lg_status dock_sites_impl(const lg_pocket* pockets, int32_t n_sites, const lg_ligands* L, const lg_dock_params* P,
                          const lg_dock_out* outs, int32_t site_major, void* stream) {
  if (!pockets || !P || !outs) return fail(LG_ERR_INVALID_ARG, "pockets, params and outs must not be NULL");
  if (n_sites < 1 || n_sites > 4096) return fail(LG_ERR_INVALID_ARG, "n_sites %d outside 1..4096", n_sites);
  for (int si = 0; si < n_sites; ++si) {
    if (!pockets[si]) return fail(LG_ERR_INVALID_ARG, "pocket %d is NULL", si);
    const lg_pocket_desc& a = pockets[0]->desc;
    const lg_pocket_desc& b = pockets[si]->desc;
    if (pockets[si]->device != pockets[0]->device || a.nx != b.nx || a.ny != b.ny || a.nz != b.nz ||
        a.spacing != b.spacing || a.inv_spacing != b.inv_spacing)
      return fail(LG_ERR_INVALID_ARG, "site %d: every site needs the first site's device, dimensions and spacing", si);
  }
  lg_status s = check_ligands(L, true);
  if (s != LG_OK) return s;
  if (P->restarts < 1 || P->restarts > LG_MAX_RESTARTS) return fail(LG_ERR_LIMIT, "restarts %d outside 1..%d", P->restarts, LG_MAX_RESTARTS);
  if (P->angle_samples < 1 || P->angle_samples > LG_MAX_SAMPLES || P->trans_samples < 1 || P->trans_samples > LG_MAX_SAMPLES)
    return fail(LG_ERR_LIMIT, "samples per scan outside 1..%d", LG_MAX_SAMPLES);
  if (P->sweeps < 0) return fail(LG_ERR_INVALID_ARG, "sweeps < 0");
  if (P->top_k < 1 || P->top_k > P->restarts) return fail(LG_ERR_INVALID_ARG, "top_k %d outside 1..R", P->top_k);
  if (!P->restart_table || !P->angle_table) return fail(LG_ERR_INVALID_ARG, "restart_table and angle_table are required");
  if (!std::isfinite(P->trans_step) || !std::isfinite(P->clash_dist2)) return fail(LG_ERR_INVALID_ARG, "non-finite step or clash distance");
  for (int si = 0; si < n_sites; ++si)
    if (L->n > 0 && (!outs[si].score || !outs[si].restart_id || !outs[si].x || !outs[si].y || !outs[si].z))
      return fail(LG_ERR_INVALID_ARG, "site %d: score, restart_id and x/y/z outputs are required", si);
  if (L->n == 0) return LG_OK;
  const int n = L->n, R = P->restarts;
  const long long moves_per_site = (long long)R * P->sweeps * (6LL * n + L->total_torsions);
  if (moves_per_site * n_sites > (1LL << 40)) return fail(LG_ERR_LIMIT, "move records of all sites too large");
  const int chunk = pockets[0]->tuning.restart_chunk;
  if ((long long)n * ((R + chunk - 1) / chunk) * n_sites >= (1LL << 30))
    return fail(LG_ERR_LIMIT, "ligands x restart chunks x sites must stay below 2^30 work items");
  lg_pocket p = pockets[0];
  hipStream_t st = (hipStream_t)stream;
  LG_HIP(hipSetDevice(p->device));
  const lg_tuning& tu = p->tuning;
  const int B = tu.n_atom_clusters * tu.n_rot_clusters;
  Layout lay;
  const size_t o_stats = lay.take(16 * sizeof(int32_t));
  const size_t o_final = lay.take((size_t)n * R * n_sites * sizeof(float));
  const size_t o_moves = lay.take((size_t)moves_per_site * n_sites * sizeof(uint16_t));
  const size_t o_cls = lay.take((size_t)n * sizeof(int32_t));
  const size_t o_perm = lay.take((size_t)n * sizeof(int32_t));
  const size_t o_cnt = lay.take((size_t)(4 * B + 1) * sizeof(int32_t));
  const size_t o_grids = lay.take((size_t)n_sites * sizeof(lg::SiteGrid));
  s = ensure_ws(p, lay.off);
  if (s != LG_OK) return s;
  char* ws = (char*)p->ws;
  int max_atoms = 0, max_tors = 0;
  s = check_on_device(p, L, (int32_t*)(ws + o_stats), st, &max_atoms, &max_tors);
  if (s != LG_OK) return s;
  std::vector<lg::SiteGrid> grids(n_sites);
  for (int si = 0; si < n_sites; ++si) {
    const lg::GridDev& g = pockets[si]->grid;
    lg::SiteGrid& sg = grids[si];
    sg.g0 = g.g0;
    sg.gb = g.gb;
    sg.gk = g.gk;
    for (int a = 0; a < 3; ++a) {
      sg.c0[a] = g.c0[a];
      sg.o[a] = g.o[a];
    }
    sg.out = g.out;
    for (int a = 0; a < 3; ++a) sg.c[a] = pockets[si]->desc.center[a];
  }
  lg::SiteGrid* dgrids = (lg::SiteGrid*)(ws + o_grids);
  LG_HIP(hipMemcpyAsync(dgrids, grids.data(), grids.size() * sizeof(lg::SiteGrid), hipMemcpyHostToDevice, st));
  LG_HIP(hipStreamSynchronize(st));

  lg::DockDev D;
  D.R = R;
  D.A = P->angle_samples;
  D.T = P->trans_samples;
  D.S = P->sweeps;
  D.delta = P->trans_step;
  D.clash2 = P->clash_dist2;
  D.clash_r2 = P->clash_dist2 > 0.f ? (std::sqrt(P->clash_dist2) + 0.05f) * (std::sqrt(P->clash_dist2) + 0.05f) : 0.f;
  for (int a = 0; a < 3; ++a) D.c[a] = p->desc.center[a];
  D.restarts = P->restart_table;
  D.angles = P->angle_table;
  D.final_scores = (float*)(ws + o_final);
  D.moves = (uint16_t*)(ws + o_moves);
  D.lazy_clash = tu.lazy_clash;
  D.trace = nullptr;
  D.trace_w = 6;
  lg::SitesDev Sd{dgrids, n_sites, site_major ? 1 : 0, (size_t)n * R, (size_t)moves_per_site};
  const lg::LigDev Lg = lig_dev(L);
  const int spl = spl_for(D.A, D.T);
  if (spl > 16) return fail(LG_ERR_LIMIT, "samples per lane %d > 16", spl);

  lg::ClusterBounds cb;
  std::memset(&cb, 0, sizeof cb);
  cb.na = tu.n_atom_clusters;
  cb.nr = tu.n_rot_clusters;
  for (int c = 0; c < cb.na; ++c) cb.atom[c] = tu.atom_bounds[c];
  for (int c = 0; c < cb.nr; ++c) cb.rot[c] = tu.rot_bounds[c];
  cb.atom[cb.na - 1] = LG_MAX_ATOMS;
  int32_t* cls = (int32_t*)(ws + o_cls);
  int32_t* perm = (int32_t*)(ws + o_perm);
  int32_t* counts = (int32_t*)(ws + o_cnt);
  int32_t* start = counts + B;
  int32_t* fill = start + B + 1;
  int32_t* cursors = fill + B;
  LG_HIP(lg::launch_bucketing(L->atom_offset, L->tors_offset, n, cb, cls, counts, start, fill, perm, cursors, st));
  // every bucket's persistent launch on the caller's stream, largest instance first
  for (int ca = cb.na - 1; ca >= 0; --ca) {
    const int nslot = std::max(1, (std::min(cb.atom[ca], max_atoms) + 63) / 64);
    const int wpb = tu.waves_per_block[nslot - 1];
    int bpc = 0;
    LG_HIP(lg::occupancy_dock_bucket(nslot, spl, wpb, p->grid.tab_len, &bpc));
    if (bpc < 1) return fail(LG_ERR_DEVICE, "kernel instance (%d slots, %d samples/lane) cannot be resident", nslot, spl);
    for (int cr = cb.nr - 1; cr >= 0; --cr) {
      lg::QueueDev Q{perm, start, cursors, ca * cb.nr + cr, tu.restart_chunk};
      LG_HIP(lg::launch_dock_sites(nslot, spl, wpb, bpc * p->cus * tu.grid_scale, p->grid, Lg, D, Q, Sd, st));
    }
  }
  const int topk_slots = std::max(1, (max_atoms + 63) / 64);
  for (int si = 0; si < n_sites; ++si) {
    lg::DockDev Ds = D;
    for (int a = 0; a < 3; ++a) Ds.c[a] = pockets[si]->desc.center[a];
    Ds.final_scores = D.final_scores + (size_t)si * Sd.scores_stride;
    Ds.moves = D.moves + (size_t)si * Sd.moves_stride;
    const lg_dock_out& O = outs[si];
    LG_HIP(lg::launch_topk(topk_slots, Lg, Ds, n, P->top_k, O.score, O.restart_id, O.x, O.y, O.z, O.all_scores,
                           O.pivot, st));
  }
  // the bucket statistics and any captured single-site batch referred to the
  // workspace contents this call replaced
  p->launches.clear();
  p->timed = false;
  if (p->gexec) {
    (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
    p->gkey.clear();
  }
  return LG_OK;
}

}  // namespace

extern "C" {

lg_status lg_dock_stream(lg_pocket p, const lg_host_ligands* H, const lg_dock_params* P, int32_t chunk,
                         const lg_host_out* O, void* stream) {
  return guarded([&] { return dock_stream_impl(p, H, P, chunk, O, stream); });
}

lg_status lg_dock_sites(const lg_pocket* pockets, int32_t n_sites, const lg_ligands* L, const lg_dock_params* P,
                        const lg_dock_out* outs, int32_t site_major, void* stream) {
  return guarded([&] { return dock_sites_impl(pockets, n_sites, L, P, outs, site_major, stream); });
}

int32_t lg_bucket_stats(lg_pocket p, lg_bucket_stat* out, int32_t capacity) {
  if (!p) return fail(LG_ERR_INVALID_ARG, "pocket is NULL");
  const int nl = (int)p->launches.size();
  if (!out || capacity <= 0 || nl == 0) return nl;
  if (hipDeviceSynchronize() != hipSuccess) return fail(LG_ERR_DEVICE, "device synchronise failed");
  int32_t counts[16 * 32] = {};   // at most 16 atom x 32 rotamer clusters
  const int nb = p->tuning.n_atom_clusters * p->tuning.n_rot_clusters;
  if (p->counts_dev &&
      hipMemcpy(counts, p->counts_dev, (size_t)nb * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(LG_ERR_DEVICE, "reading bucket counts failed");
  for (int l = 0; l < nl && l < capacity; ++l) {
    out[l] = p->launches[l];
    if (p->launches[l].bucket < nb) out[l].ligands = counts[p->launches[l].bucket];
    float ms = -1.f, span = -1.f;
    if (p->timed && (hipEventElapsedTime(&ms, p->events[1 + 2 * l], p->events[2 + 2 * l]) != hipSuccess ||
                     hipEventElapsedTime(&span, p->events[0], p->events[1 + 2 * nl]) != hipSuccess)) {
      (void)hipGetLastError();
      ms = span = -1.f;
    }
    out[l].ms = ms;
    out[l].span_ms = span;
  }
  return nl;
}

lg_status lg_autotune(lg_pocket p, const lg_ligands* L, const lg_dock_params* P, int32_t passes, lg_tuning* out,
                      float* best_ms, void* stream) {
  if (!p || !P || !out) return fail(LG_ERR_INVALID_ARG, "pocket, params and out must not be NULL");
  lg_status s = check_ligands(L, true);
  if (s != LG_OK) return s;
  if (L->n < 1) return fail(LG_ERR_INVALID_ARG, "the tuning sample is empty");
  if (passes < 1 || passes > 8) return fail(LG_ERR_INVALID_ARG, "passes %d outside 1..8", passes);
  if (P->top_k < 1 || P->top_k > P->restarts) return fail(LG_ERR_INVALID_ARG, "top_k %d outside 1..R", P->top_k);
  hipStream_t st = (hipStream_t)stream;
  LG_HIP(hipSetDevice(p->device));

  // largest ligand and bond count of the sample
  Layout lay;
  const size_t o_stats = lay.take(16 * sizeof(int32_t));
  s = ensure_ws(p, lay.off);
  if (s != LG_OK) return s;
  int max_atoms = 0, max_tors = 0;
  s = check_on_device(p, L, (int32_t*)((char*)p->ws + o_stats), st, &max_atoms, &max_tors);
  if (s != LG_OK) return s;

  // outputs of the trial calls
  const size_t nk = (size_t)L->n * P->top_k, ak = (size_t)L->total_atoms * P->top_k;
  void* buf = nullptr;
  if (hipMalloc(&buf, (nk * 5 + 3 * ak) * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LG_ERR_OUT_OF_MEMORY, "autotuner outputs could not be allocated");
  }
  float* f = (float*)buf;
  lg_dock_out O;
  std::memset(&O, 0, sizeof O);
  O.score = f;
  O.restart_id = (int32_t*)(f + nk);
  O.pivot = f + 2 * nk;
  O.x = f + 5 * nk;
  O.y = O.x + ak;
  O.z = O.y + ak;
  lg_dock_params tp = *P;
  tp.mode = LG_BUCKETED;
  const lg_tuning saved = p->tuning;

  // time of the bucket launches of one call (events recorded between them), best of two
  auto trial = [&](lg_tuning t, float* ms) -> lg_status {
    t.use_graph = 0;
    lg_status r = lg_set_tuning(p, &t);
    if (r != LG_OK) return r;
    float best = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      r = lg_dock_batch(p, L, &tp, &O, stream);
      if (r != LG_OK) return r;
      LG_HIP(hipStreamSynchronize(st));
      float m = 0.f;
      LG_HIP(hipEventElapsedTime(&m, p->events[0], p->events[1 + 2 * p->launches.size()]));
      best = std::min(best, m);
    }
    *ms = best;
    return LG_OK;
  };

  lg_tuning cur = saved;
  float cur_ms = 0.f;
  s = trial(cur, &cur_ms);
  // a candidate replaces the current choice only if it is at least 1 % faster
  auto consider = [&](const lg_tuning& t) -> lg_status {
    float ms = 0.f;
    lg_status r = trial(t, &ms);
    if (r == LG_OK && ms < 0.99f * cur_ms) {
      cur = t;
      cur_ms = ms;
    }
    return r;
  };
  for (int pass = 0; pass < passes && s == LG_OK; ++pass) {
    // size buckets: one cluster per kernel instance (atom slots), with or without
    // rotamer clusters, or one cluster for everything
    {
      lg_tuning t = cur;
      t.n_atom_clusters = lg_atom_clusters(4, 64, std::max(max_atoms, 1), t.atom_bounds);
      t.n_rot_clusters = 1;
      t.rot_bounds[0] = LG_MAX_TORSIONS;
      if (s == LG_OK) s = consider(t);
      t.n_rot_clusters = lg_rotamer_clusters(4, std::max(max_tors, 1), t.rot_bounds);
      if (s == LG_OK && t.n_rot_clusters > 1) s = consider(t);
      t.n_atom_clusters = 1;
      t.atom_bounds[0] = LG_MAX_ATOMS;
      t.n_rot_clusters = 1;
      t.rot_bounds[0] = LG_MAX_TORSIONS;
      if (s == LG_OK) s = consider(t);
    }
    // wavefronts per block of each kernel instance in use
    for (int slots = 1; slots <= (max_atoms + 63) / 64 && s == LG_OK; ++slots)
      for (int w : {1, 2, 4}) {
        if (w == cur.waves_per_block[slots - 1] || s != LG_OK) continue;
        lg_tuning t = cur;
        t.waves_per_block[slots - 1] = w;
        s = consider(t);
      }
    for (int c : {2, 4, 8, 16, 32}) {
      if (c == cur.restart_chunk || c > P->restarts || s != LG_OK) continue;
      lg_tuning t = cur;
      t.restart_chunk = c;
      s = consider(t);
    }
    for (int g : {1, 2, 4}) {
      if (g == cur.grid_scale || s != LG_OK) continue;
      lg_tuning t = cur;
      t.grid_scale = g;
      s = consider(t);
    }
    if (s == LG_OK) {
      lg_tuning t = cur;
      t.lazy_clash = 1 - cur.lazy_clash;
      s = consider(t);
    }
  }
  (void)hipFree(buf);
  if (s != LG_OK) {
    p->tuning = saved;
    return s;
  }
  cur.use_graph = saved.use_graph;
  lg_status r = lg_set_tuning(p, &cur);
  if (r != LG_OK) return r;
  *out = cur;
  if (best_ms) *best_ms = cur_ms;
  return LG_OK;
}

lg_status lg_score(lg_pocket p, const lg_ligands* L, int32_t interp, const float* moves, float* score, float* grad,
                   int32_t top_m, int32_t* top_idx, float* top_score, void* stream) {
  if (!p) return fail(LG_ERR_INVALID_ARG, "pocket is NULL");
  lg_status s = check_ligands(L, grad != nullptr || moves != nullptr);
  if (s != LG_OK) return s;
  if (interp != LG_NEAREST && interp != LG_TRILINEAR) return fail(LG_ERR_INVALID_ARG, "interp must be LG_NEAREST or LG_TRILINEAR");
  if ((grad || moves) && interp != LG_TRILINEAR) return fail(LG_ERR_INVALID_ARG, "gradients and moves need LG_TRILINEAR");
  if (L->n > 0 && !score) return fail(LG_ERR_INVALID_ARG, "score is NULL");
  if (top_m < 0 || top_m > L->n) return fail(LG_ERR_INVALID_ARG, "top_m %d outside 0..n", top_m);
  if (top_m > 0 && (!top_idx || !top_score)) return fail(LG_ERR_INVALID_ARG, "top_idx and top_score are required for top_m > 0");
  if (L->n == 0) return LG_OK;
  hipStream_t st = (hipStream_t)stream;
  LG_HIP(hipSetDevice(p->device));
  const int n = L->n;
  Layout lay;
  const size_t o_stats = lay.take(16 * sizeof(int32_t));
  const size_t o_rank = top_m > 0 ? lay.take(lg::rank_scratch_bytes(n, top_m)) : 0;
  s = ensure_ws(p, lay.off);
  if (s != LG_OK) return s;
  int max_atoms = 0, max_tors = 0;
  host_maxima(L, &max_atoms, &max_tors);
  if (max_atoms < 0) {
    s = check_on_device(p, L, (int32_t*)((char*)p->ws + o_stats), st, &max_atoms, &max_tors);
    if (s != LG_OK) return s;
  }
  if (moves)
    LG_HIP(lg::launch_score_moves((max_atoms + 63) / 64, p->grid, lig_dev(L), moves, n, score, grad, st));
  else
    LG_HIP(lg::launch_score(p->grid, lig_dev(L), n, interp, score, grad, st));
  if (top_m > 0)
    LG_HIP(lg::launch_rank(score, n, 1, top_m, (char*)p->ws + o_rank, top_idx, top_score, nullptr, st));
  return LG_OK;
}

lg_status lg_rank(lg_pocket p, const float* score, int32_t n_groups, int32_t group_size, int32_t top_m,
                  int32_t* top_idx, float* top_score, int32_t* top_member, void* stream) {
  if (!p) return fail(LG_ERR_INVALID_ARG, "pocket is NULL");
  if (n_groups < 0 || group_size < 1) return fail(LG_ERR_INVALID_ARG, "n_groups %d < 0 or group_size %d < 1", n_groups, group_size);
  if ((long long)n_groups * group_size > INT32_MAX) return fail(LG_ERR_LIMIT, "n_groups * group_size exceeds 2^31 - 1");
  if (top_m < 0 || top_m > n_groups) return fail(LG_ERR_INVALID_ARG, "top_m %d outside 0..n_groups", top_m);
  if (n_groups > 0 && !score) return fail(LG_ERR_INVALID_ARG, "score is NULL");
  if (top_m > 0 && (!top_idx || !top_score)) return fail(LG_ERR_INVALID_ARG, "top_idx and top_score are required for top_m > 0");
  if (top_m == 0) return LG_OK;
  hipStream_t st = (hipStream_t)stream;
  LG_HIP(hipSetDevice(p->device));
  lg_status s = ensure_ws(p, lg::rank_scratch_bytes(n_groups, top_m));
  if (s != LG_OK) return s;
  LG_HIP(lg::launch_rank(score, n_groups, group_size, top_m, p->ws, top_idx, top_score, top_member, st));
  return LG_OK;
}

lg_status lg_rank_static(const float* score, int32_t n_groups, int32_t group_size, int32_t top_m,
                         int32_t* top_idx, float* top_score, int32_t* top_member, void* stream) {
  if (n_groups < 0 || group_size < 1) return fail(LG_ERR_INVALID_ARG, "n_groups %d < 0 or group_size %d < 1", n_groups, group_size);
  if ((long long)n_groups * group_size > INT32_MAX) return fail(LG_ERR_LIMIT, "n_groups * group_size exceeds 2^31 - 1");
  if (top_m < 0 || top_m > n_groups) return fail(LG_ERR_INVALID_ARG, "top_m %d outside 0..n_groups", top_m);
  if (n_groups > LG_RANK_STATIC_MAX_GROUPS || top_m > LG_RANK_STATIC_MAX_TOP)
    return fail(LG_ERR_LIMIT, "n_groups %d or top_m %d above the fixed scratch's %d / %d", n_groups, top_m,
                LG_RANK_STATIC_MAX_GROUPS, LG_RANK_STATIC_MAX_TOP);
  if (n_groups > 0 && !score) return fail(LG_ERR_INVALID_ARG, "score is NULL");
  if (top_m > 0 && (!top_idx || !top_score)) return fail(LG_ERR_INVALID_ARG, "top_idx and top_score are required for top_m > 0");
  if (top_m == 0) return LG_OK;
  void* work = nullptr;
  size_t bytes = 0;
  LG_HIP(lg::rank_static_scratch(&work, &bytes));
  if (lg::rank_scratch_bytes(n_groups, top_m) > bytes)
    return fail(LG_ERR_LIMIT, "ranking needs %zu bytes of scratch, the fixed array holds %zu",
                lg::rank_scratch_bytes(n_groups, top_m), bytes);
  LG_HIP(lg::launch_rank(score, n_groups, group_size, top_m, work, top_idx, top_score, top_member,
                         (hipStream_t)stream));
  return LG_OK;
}

lg_status lg_refine(lg_pocket p, const lg_ligands* L, const lg_refine_params* rp, float* x_out, float* y_out,
                    float* z_out, float* score_out, void* stream) {
  if (!p || !rp) return fail(LG_ERR_INVALID_ARG, "pocket and params must not be NULL");
  lg_status s = check_ligands(L, true);
  if (s != LG_OK) return s;
  if (rp->steps < 0 || rp->steps > 100000) return fail(LG_ERR_LIMIT, "steps %d outside 0..100000", rp->steps);
  const float quarter = 0.78539816f;
  if (!std::isfinite(rp->eta_t) || !std::isfinite(rp->eta_w) || !std::isfinite(rp->eta_th) ||
      !std::isfinite(rp->clash_dist2) || !(rp->clip_t > 0.f) || !std::isfinite(rp->clip_t) ||
      !(rp->clip_w > 0.f) || rp->clip_w > quarter || !(rp->clip_th > 0.f) || rp->clip_th > quarter)
    return fail(LG_ERR_INVALID_ARG, "steps need finite etas, clip_t > 0 and rotation clips in (0, pi/4]");
  if (rp->poses_per_ligand < 1) return fail(LG_ERR_INVALID_ARG, "poses_per_ligand %d < 1", rp->poses_per_ligand);
  if ((long long)L->n * rp->poses_per_ligand > INT32_MAX / 64 ||
      (long long)L->total_atoms * rp->poses_per_ligand > INT32_MAX)
    return fail(LG_ERR_LIMIT, "n * poses_per_ligand or total_atoms * poses_per_ligand too large");
  if (L->n > 0 && (!x_out || !y_out || !z_out || !score_out)) return fail(LG_ERR_INVALID_ARG, "outputs are required");
  if (L->n == 0) return LG_OK;
  hipStream_t st = (hipStream_t)stream;
  LG_HIP(hipSetDevice(p->device));
  const int n = L->n;
  // size classes: ligands of at most 32 atoms and 31 bonds with two or more
  // poses each are refined two poses per wavefront (a half-wavefront has a lane
  // per bond and one for the rigid rotation); the others by the instance with
  // one atom slot per 64 atoms.  Class (atom class c, bond class r) is bucket
  // c * nr + r.
  const bool pairs = rp->poses_per_ligand >= 2;
  lg::ClusterBounds cb;
  std::memset(&cb, 0, sizeof cb);
  cb.na = 0;
  if (pairs) cb.atom[cb.na++] = 32;
  for (int c = 0; c < LG_MAX_ATOMS / 64; ++c) cb.atom[cb.na++] = 64 * (c + 1);
  cb.nr = pairs ? 2 : 1;
  cb.rot[0] = pairs ? LG_MAX_TORSIONS - 1 : LG_MAX_TORSIONS;
  cb.rot[1] = LG_MAX_TORSIONS;
  const int nb = cb.na * cb.nr;
  Layout lay;
  const size_t o_stats = lay.take(16 * sizeof(int32_t));
  const size_t o_cls = lay.take((size_t)n * sizeof(int32_t));
  const size_t o_perm = lay.take((size_t)n * sizeof(int32_t));
  const size_t o_cnt = lay.take((size_t)(4 * nb + 1) * sizeof(int32_t));
  s = ensure_ws(p, lay.off);
  if (s != LG_OK) return s;
  char* ws = (char*)p->ws;
  int max_atoms = 0, max_tors = 0;
  host_maxima(L, &max_atoms, &max_tors);
  if (max_atoms < 0) {
    s = check_on_device(p, L, (int32_t*)(ws + o_stats), st, &max_atoms, &max_tors);
    if (s != LG_OK) return s;
  }
  lg::RefineDev R;
  R.lig_ids = nullptr;
  R.steps = rp->steps;
  R.kpl = rp->poses_per_ligand;
  R.eta_t = rp->eta_t; R.eta_w = rp->eta_w; R.eta_th = rp->eta_th;
  R.clip_t = rp->clip_t; R.clip_w = rp->clip_w; R.clip_th = rp->clip_th;
  R.clash2 = rp->clash_dist2;
  R.xo = x_out; R.yo = y_out; R.zo = z_out; R.score = score_out;
  const int kpl = rp->poses_per_ligand;
  if (pairs && max_atoms <= 32 && max_tors >= 0 && max_tors < LG_MAX_TORSIONS) {
    LG_HIP(lg::launch_refine_pair(p->grid, lig_dev(L), R, n, st));
    return LG_OK;
  }
  if (!pairs && max_atoms <= 64) {
    LG_HIP(lg::launch_refine(1, p->grid, lig_dev(L), R, n * kpl, st));
    return LG_OK;
  }
  // ligands grouped by size class, each class refined by the instance that fits it
  int32_t* cls = (int32_t*)(ws + o_cls);
  int32_t* perm = (int32_t*)(ws + o_perm);
  int32_t* counts = (int32_t*)(ws + o_cnt);
  int32_t* start = counts + nb;
  int32_t* fill = start + nb + 1;
  int32_t* cursors = fill + nb;
  LG_HIP(lg::launch_bucketing(L->atom_offset, L->tors_offset, n, cb, cls, counts, start, fill, perm, cursors, st));
  int32_t hs[2 * (LG_MAX_ATOMS / 64 + 1) + 1];
  LG_HIP(hipMemcpyAsync(hs, start, (size_t)(nb + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  LG_HIP(hipStreamSynchronize(st));
  for (int b = 0; b < nb; ++b) {
    const int cnt = hs[b + 1] - hs[b];
    if (cnt <= 0) continue;
    const int c = b / cb.nr, r = b % cb.nr;
    R.lig_ids = perm + hs[b];
    if (pairs && c == 0 && r == 0)
      LG_HIP(lg::launch_refine_pair(p->grid, lig_dev(L), R, cnt, st));
    else
      LG_HIP(lg::launch_refine((cb.atom[c] + 63) / 64, p->grid, lig_dev(L), R, cnt * kpl, st));
  }
  return LG_OK;
}

lg_status lg_valu_probe(lg_pocket p, int32_t kind, int32_t iters, double* lane_ops_per_s, void* stream) {
  if (!p || !lane_ops_per_s) return fail(LG_ERR_INVALID_ARG, "pocket and lane_ops_per_s must not be NULL");
  if (kind < 0 || kind > 6) return fail(LG_ERR_INVALID_ARG, "kind %d outside 0..6", kind);
  if (iters < 1 || iters > 1000000) return fail(LG_ERR_LIMIT, "iters %d outside 1..1000000", iters);
  hipStream_t st = (hipStream_t)stream;
  LG_HIP(hipSetDevice(p->device));
  const int blocks = p->cus * 8;   // eight 4-wavefront blocks per CU: eight wavefronts per SIMD
  float* out = nullptr;
  if (hipMalloc((void**)&out, (size_t)blocks * 256 * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LG_ERR_OUT_OF_MEMORY, "probe buffer could not be allocated");
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float ms = 0.f;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = lg::launch_valu_probe(kind, blocks, iters, out, st);   // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  if (e == hipSuccess) e = lg::launch_valu_probe(kind, blocks, iters, out, st);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(out);
  if (e != hipSuccess) return fail(LG_ERR_DEVICE, "probe failed: %s", hipGetErrorString(e));
  const double ops_per_iter = kind == 6 ? 80.0 : 8.0;   // kind 6: ten VALU operations per chain step
  *lane_ops_per_s = ops_per_iter * iters * (double)blocks * 256.0 / (ms * 1e-3);
  return LG_OK;
}

}  // extern "C"
