/*
 * lg.h -- C ABI of the MI355X docking hot path.
 *
 * The calls follow the paper's statement of the virtual-screening problem
 * (Sec. 2): identify a docking site (lg_load_pocket), dock every ligand of a
 * bucket into it, i.e. estimate the 3D placement of its atoms
 * (lg_dock_batch; lg_dock_stream for a library held in host memory,
 * lg_dock_sites for several docking sites of one target), evaluate the
 * interaction strength (lg_score), refine the best poses locally (lg_refine)
 * and rank the library (lg_rank).  Buckets of ligands of similar
 * atom and rotamer counts, each docked by a kernel instantiated for its size
 * class with a bucket size derived from occupancy, are the paper's
 * out-of-kernel optimisation (Sec. 3, Eq. 1); lg_dock_batch with LG_BUCKETED is
 * its GPU-side form, and lg_autotune picks its buckets and kernel shapes by
 * measurement.
 *
 * Conventions (all entry points):
 *  - Pointers marked "device" are device memory; "host" are host memory.
 *    The caller owns every array it passes; the library never frees them.
 *  - Work is enqueued on `stream` (a hipStream_t, NULL = default stream) and is
 *    asynchronous: keep buffers alive until the stream has completed.
 *  - Every call returns an lg_status; nothing throws across the ABI and
 *    nothing aborts.  Argument and limit checks are synchronous and return
 *    before any work is enqueued.  Ligand data is checked on the host when the
 *    batch carries host copies of its offsets and bond atoms (lg_ligands), and
 *    the call then enqueues without waiting on the stream; otherwise a small
 *    kernel checks the device copies and its counters are read back before the
 *    docking work (one stream synchronisation).
 *    HIP errors map to LG_ERR_DEVICE and are reported by the call that
 *    observes them; a host allocation the library cannot make (its staging,
 *    plans, chunk lists) returns LG_ERR_OUT_OF_MEMORY.  lg_last_error() gives
 *    a message (at most 511 characters) for the last failing call of the
 *    calling thread.
 *  - Coordinates are Angstrom, FP32.  Arithmetic is FP32 with explicit fma
 *    (no contraction); given the same inputs, results are bitwise
 *    reproducible run to run and identical between LG_PLAIN and LG_BUCKETED.
 */
#ifndef LG_H_
#define LG_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LG_OK = 0,
  LG_ERR_INVALID_ARG = -1,   /* null pointer, bad size, inconsistent offsets */
  LG_ERR_LIMIT = -2,         /* a size beyond the limits below */
  LG_ERR_OUT_OF_MEMORY = -3, /* device workspace could not be allocated */
  LG_ERR_DEVICE = -4,        /* a HIP call failed */
  LG_ERR_UNSUPPORTED = -5    /* no gfx950 device, or an unsupported option */
} lg_status;

enum { LG_NEAREST = 0, LG_TRILINEAR = 1 };
enum { LG_PLAIN = 0, LG_BUCKETED = 1 };

#define LG_MAX_ATOMS 256      /* atoms per ligand */
#define LG_MAX_TORSIONS 32    /* rotatable bonds per ligand (frag_mask width) */
#define LG_MAX_SAMPLES 1024   /* angle or translation samples per scan */
#define LG_MAX_RESTARTS 65536

/* Docking site (Sec. 2): a node-centred grid of float32 values, x fastest,
 * node (ix,iy,iz) at origin + (ix,iy,iz)*spacing.  Nearest lookups take node
 * (int)f per axis with f = fma(x, inv_spacing, c), c = fma(-origin,
 * inv_spacing, 0.5) (FP32), when 0 <= f < n on every axis; trilinear lookups
 * need 0 <= (x - origin)*inv_spacing < n-1 on every axis.  Positions outside either rule score out_value (zero gradient).
 * Restart offsets are relative to `center`. */
typedef struct {
  int32_t nx, ny, nz;        /* 2..1024 each; (nx+2)(ny+2) < 2^21 and (nx+2)(ny+2)(nz+2) < 2^29 */
  float spacing;             /* Angstrom, > 0 */
  float inv_spacing;         /* the FP32 value of 1/spacing every lookup uses */
  float origin[3];
  float center[3];
  float out_value;
} lg_pocket_desc;

typedef struct lg_pocket_s* lg_pocket;

/* A batch of ligands (or of poses of ligands), CSR + SoA.  Ligand i owns atoms
 * [atom_offset[i], atom_offset[i+1]) and rotatable bonds [tors_offset[i],
 * tors_offset[i+1]).  Rotamers (Sec. 3) are the moving fragments F_k: bit k of
 * frag_mask[a] says that atom a moves with bond k; F_k holds the moving-side
 * atom b_k.  Bond k is (a_k, b_k) = (static-side atom, moving-side atom), local
 * atom ids.  Bonds are scanned in the order given.
 *   n                 number of ligands (0 is allowed: nothing to do)
 *   total_atoms       host value = atom_offset[n]
 *   total_torsions    host value = tors_offset[n]
 *   atom_offset_host  optional host copies of the offsets and of the bond atoms,
 *   tors_offset_host  each checked on the host before any launch (sizes, limits,
 *   tors_atoms_host   totals, bond ids).  They must equal the device arrays.
 *                     With all three, lg_dock_batch, lg_score and lg_refine
 *                     take the batch's sizes from them and do not read device
 *                     data back (lg_dock_batch and lg_score then return without
 *                     waiting on the stream).  Without all three, the call
 *                     checks the device copies with one small kernel and a
 *                     synchronous read-back of its counters (sizes, limits,
 *                     consistency, local ids).  Either way bad data is reported
 *                     as LG_ERR_INVALID_ARG / LG_ERR_LIMIT, never docked.
 * Limits: 1 <= atoms <= LG_MAX_ATOMS and 0 <= bonds <= LG_MAX_TORSIONS per
 * ligand; a bond's two atoms are distinct local ids; total_atoms <= 2^30 - 256
 * per batch (the kernels address the atom arrays with 32-bit byte offsets). */
typedef struct {
  int32_t n;
  int32_t total_atoms;
  int32_t total_torsions;
  const int32_t* atom_offset;      /* device [n+1] */
  const int32_t* tors_offset;      /* device [n+1] */
  const float* x;                  /* device [total_atoms] */
  const float* y;
  const float* z;
  const uint32_t* frag_mask;       /* device [total_atoms] */
  const int32_t* tors_atoms;       /* device [2*total_torsions] (a_k, b_k) */
  const float* inv_bond_len;       /* device [total_torsions] FP32 of 1/|x_b - x_a| of the input */
  const float* ref_point;          /* device [3n] rigid-body pivot P0 (e.g. the centroid) */
  const int32_t* atom_offset_host; /* host [n+1] or NULL */
  const int32_t* tors_offset_host; /* host [n+1] or NULL */
  const int32_t* tors_atoms_host;  /* host [2*total_torsions] or NULL (needs the two above) */
} lg_ligands;

/* Docking parameters.  Per restart r the ligand is placed at
 * M_r (x0 - P0) + center + t_r, then `sweeps` times: rotation scans about the
 * lab x, y, z axes through the pivot, translation scans along x, y, z, then a
 * greedy scan of every rotatable bond with an intramolecular clash check.
 * Sample j of a rotation or torsion scan turns by 2*pi*j/A (angle_table row j);
 * sample j of a translation scan shifts by trans_step*(j < T/2 ? j : j - T).
 * Sample 0 is the current pose.  Each scan keeps its best admissible sample
 * (nearest-voxel score sum; equal scores keep the lowest j).  A torsion sample
 * is admissible when every pair (moving atom of F_k other than b_k, atom
 * outside F_k other than a_k) is at squared distance >= clash_dist2.  The final
 * score of a restart is the trilinear score sum in atom order; the top_k
 * restarts by final score (equal scores: lower r) are returned. */
typedef struct {
  int32_t restarts;          /* R, 1..LG_MAX_RESTARTS */
  int32_t angle_samples;     /* A, 1..LG_MAX_SAMPLES */
  int32_t trans_samples;     /* T, 1..LG_MAX_SAMPLES */
  int32_t sweeps;            /* S, >= 0 */
  int32_t top_k;             /* 1..R */
  int32_t mode;              /* LG_PLAIN (one launch per ligand) or LG_BUCKETED */
  float trans_step;          /* Angstrom */
  float clash_dist2;         /* squared Angstrom */
  const float* restart_table;/* device [R][12]: row-major rotation, then offset */
  const float* angle_table;  /* device [A][2]: (cos, sin) of 2*pi*j/A */
} lg_dock_params;

/* Docking outputs (device).  Rank q of ligand i: score[i*top_k + q],
 * restart_id[i*top_k + q]; its pose atom a (local id) sits at
 * top_k*atom_offset[i] + q*N_i + a of x/y/z.  Optional: all_scores [n*R] final
 * score of every restart; trace [n][R][sweeps][6+trace_kmax] the selected
 * sample of every scan (rotations x,y,z, translations x,y,z, bonds in order;
 * unused columns untouched), with trace_kmax >= the largest bond count. */
typedef struct {
  float* score;
  int32_t* restart_id;
  float* x;
  float* y;
  float* z;
  float* all_scores;         /* optional */
  int16_t* trace;            /* optional */
  int32_t trace_kmax;
  float* pivot;              /* optional [n*top_k*3]: rigid-body pivot of each kept pose
                                (ref_point carried through placement and translations),
                                the pivot lg_refine rotates about */
} lg_dock_out;

/* Load a docking site: copies the grid (host or device memory, per
 * grid_is_device) into a library-owned device copy kept for the handle's
 * life.  *out receives the handle; the call synchronises `stream`. */
lg_status lg_load_pocket(const lg_pocket_desc* desc, const float* grid, int32_t grid_is_device,
                         void* stream, lg_pocket* out);

/* Free a handle, its grid copy and its workspace (after synchronising the
 * device).  NULL is a no-op. */
lg_status lg_free_pocket(lg_pocket pocket);

/* Dock a batch of ligands (Sec. 2 "dock", Sec. 3 buckets).  LG_PLAIN launches
 * one kernel per ligand sized for the largest class; LG_BUCKETED classifies
 * ligands on the device by (atoms, bonds) into size buckets, docks every bucket
 * in one persistent launch of its class kernel pulling (ligand, restart) items
 * from a device queue, and replays the whole sequence as one HIP graph.  Every
 * restart records its final score and the selected sample of each scan; the
 * kept poses are rebuilt from those records.  Workspace: 4 n R bytes of scores
 * plus 2 R sweeps (6 n + total_torsions) bytes of records, held by the pocket
 * handle (growing it waits for the device): calls on one handle must not
 * overlap.  LG_BUCKETED needs n * ceil(R / restart_chunk) < 2^30 work items
 * (else LG_ERR_LIMIT before any launch). */
lg_status lg_dock_batch(lg_pocket pocket, const lg_ligands* ligands, const lg_dock_params* params,
                        const lg_dock_out* out, void* stream);

/* Dock a batch into several docking sites at once (Sec. 2: a docking site is
 * one region of the target that ligands are docked into; the bucket-size
 * experiments of Sec. 5.2 dock every ligand into twelve sites of one target):
 * every ligand is docked into every site, results as lg_dock_batch with
 * LG_BUCKETED on each site in turn (outs[s] receives site s; mode and trace
 * are ignored).  The sites must share the first site's device, grid
 * dimensions and spacing (their grids, origins, centres and far values may
 * differ); the first handle's tuning and workspace are used, the workspace
 * holding the final scores and move records of every site.
 * Work items are (site, ligand, restart chunk): site_major != 0 takes the
 * sites one after another, so the caches hold about one site's grid at a time;
 * 0 interleaves the sites per ligand.  Calls on the first handle must not
 * overlap; synchronises `stream` once (validation and the site table). */
lg_status lg_dock_sites(const lg_pocket* pockets, int32_t n_sites, const lg_ligands* ligands,
                        const lg_dock_params* params, const lg_dock_out* outs, int32_t site_major, void* stream);

/* A library held in host memory: the lg_ligands layout with every array a
 * host pointer (no device copy needed). */
typedef struct {
  int32_t n;
  int32_t total_atoms;
  int32_t total_torsions;
  const int32_t* atom_offset;      /* host [n+1] */
  const int32_t* tors_offset;      /* host [n+1] */
  const float* x;                  /* host [total_atoms] */
  const float* y;
  const float* z;
  const uint32_t* frag_mask;       /* host [total_atoms] */
  const int32_t* tors_atoms;       /* host [2*total_torsions] */
  const float* inv_bond_len;       /* host [total_torsions] */
  const float* ref_point;          /* host [3n] */
} lg_host_ligands;

/* Host outputs of lg_dock_stream, in the lg_dock_out layout (pivot optional).
 * chunk_done (optional, host [ceil(n / chunk)]) is a resume manifest: chunks
 * whose entry is non-zero are skipped and their outputs left untouched; every
 * other chunk gets entry 1 once its outputs have been written to the arrays
 * above (the entry is stored after them).  With outputs and manifest in
 * persistent memory (memory-mapped files), a screen interrupted part-way is
 * completed by calling again with the same arrays; flushing them to storage
 * is the caller's business. */
typedef struct {
  float* score;                    /* host [n*top_k] */
  int32_t* restart_id;             /* host [n*top_k] */
  float* x;                        /* host [top_k*total_atoms] */
  float* y;
  float* z;
  float* pivot;                    /* host [n*top_k*3] or NULL */
  int32_t* chunk_done;             /* host [ceil(n/chunk)] or NULL */
} lg_host_out;

/* Dock a library held in host memory, streamed through the device in chunks of
 * at most `chunk` consecutive ligands -- the worker / double-buffer structure of
 * Sec. 2 on one GPU: while chunk c docks on `stream` (bucketed, launched
 * directly), chunk c+1's inputs are packed into pinned staging and copied in on
 * a copy stream and chunk c-1's results copied back on another, two buffer
 * slots alternating.  Device memory is bounded by the chunk (two slots plus the
 * docking workspace of one chunk), not by the library.  The library is
 * validated on the host first (same rules as lg_dock_batch's device check).
 * Results are those of lg_dock_batch on the whole library in LG_BUCKETED mode;
 * params' tables are device memory.  Returns when every result is in `out`.
 * Calls on one handle must not overlap.  On an error after some chunks, those
 * chunks' outputs and manifest entries are complete and the others untouched,
 * so a call with the same arrays resumes.  For tests of that path, the
 * environment variable LG_FAULT_AFTER_CHUNKS=k stops a call with LG_ERR_DEVICE
 * after k chunks; LG_WORKSPACE_LIMIT (bytes) caps the docking workspace of a
 * handle and the stream buffers (LG_ERR_OUT_OF_MEMORY above it, before any
 * work). */
lg_status lg_dock_stream(lg_pocket pocket, const lg_host_ligands* ligands, const lg_dock_params* params,
                         int32_t chunk, const lg_host_out* out, void* stream);

/* Score poses (Sec. 2 "evaluate the interaction strength", "rank").  Each
 * ligand of `poses` is one pose.  interp = LG_NEAREST or LG_TRILINEAR; score[i]
 * = sum over its atoms in atom order.  grad (optional, trilinear only): per
 * pose 6+K_i values at 6*i + tors_offset[i]: d(score)/d(t[3], omega[3],
 * theta[K]) at zero for the local move (torsions about the current bond axes,
 * rotation omega about ref_point, translation t), i.e. sum g, sum (x-P) x g,
 * u_k . sum_{F_k} (x - x_{a_k}) x g with g the trilinear gradient and u_k the
 * unit bond axis.  moves (optional, trilinear only, same layout as grad): each
 * pose is first moved by its local parameters q = (t, omega, theta) --
 * torsions in reverse bond order (k = K-1 .. 0, deepest first when bonds are
 * listed parents first) about the current bond axes, rotation by |omega| about
 * omega/|omega| through ref_point, translation (pivot included) -- then scored;
 * grad is then d(score)/dq at q (the omega part through the transposed left
 * Jacobian of SO(3)).  top_m > 0: top_idx / top_score (device [top_m]) receive
 * the global ranking (score descending, equal scores: lower index). */
lg_status lg_score(lg_pocket pocket, const lg_ligands* poses, int32_t interp, const float* moves, float* score,
                   float* grad, int32_t top_m, int32_t* top_idx, float* top_score, void* stream);

/* Local refinement of poses by gradient ascent on the trilinear score.  Each
 * step: gradient at the current pose, step = (eta_t*g_t, eta_w*g_w,
 * eta_th*g_th) clipped to norm clip_t, norm clip_w and per-bond clip_th,
 * applied as the local move of lg_score; a step that makes an intramolecular
 * clash (any pair separated by a rotatable bond, other than the bond's own
 * axis atoms, closer than sqrt(clash_dist2)) is rejected, the pose kept and
 * the step scale of later steps halved.  The best-scoring pose seen (including
 * the input) is written to x/y/z_out in the layout of the input coordinates,
 * its score to score_out [n*k].  One wavefront refines one pose; with k >= 2,
 * ligands of at most 32 atoms are refined two poses per wavefront (same
 * arithmetic per pose).  When the batch mixes size classes the call reads the
 * class counts back, which synchronises `stream`. */
typedef struct {
  int32_t steps;
  float eta_t, eta_w, eta_th;
  float clip_t, clip_w, clip_th;  /* clip_w and clip_th in (0, pi/4] */
  float clash_dist2;
  int32_t poses_per_ligand;       /* k >= 1.  k = 1: entry i of `poses` is one pose.  k > 1:
                                     x/y/z hold k poses per ligand in the lg_dock_out layout
                                     (pose q of ligand i at k*atom_offset[i] + q*N_i) and
                                     ref_point holds one pivot per pose [3*(k*i + q)] */
} lg_refine_params;

lg_status lg_refine(lg_pocket pocket, const lg_ligands* poses, const lg_refine_params* params,
                    float* x_out, float* y_out, float* z_out, float* score_out, void* stream);

/* Rank a library (Sec. 2 "rank the input chemical library"): score holds
 * group_size consecutive values per ligand (device [n_groups*group_size], e.g.
 * lg_refine's scores of a ligand's k poses); each ligand is ranked by its best
 * value (equal values within a ligand: lower member).  top_idx / top_score
 * (device [top_m]) receive the top_m ligands, best first, equal scores ordered
 * by lower ligand index; top_member (optional, device [top_m]) the member that
 * gave each ligand its score.  Uses the handle's workspace: calls on one handle
 * must not overlap. */
lg_status lg_rank(lg_pocket pocket, const float* score, int32_t n_groups, int32_t group_size, int32_t top_m,
                  int32_t* top_idx, float* top_score, int32_t* top_member, void* stream);

/* lg_rank for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): same
 * arguments and results as lg_rank, no pocket handle, and no allocation of any
 * kind.  Its scratch is a fixed device array in the library (about 12 MiB,
 * one copy per device, held until the process ends), looked up on the first
 * call on each device; the device is the caller's current device, which must
 * own `stream` and the buffers.  Limits: n_groups <= LG_RANK_STATIC_MAX_GROUPS
 * and top_m <= LG_RANK_STATIC_MAX_TOP, else LG_ERR_LIMIT before any device
 * work.  Every call on one device shares that array (each call re-initialises
 * what it reads, on `stream`): calls that overlap on one device -- concurrent
 * streams or threads -- race and give wrong results; serialise them. */
#define LG_RANK_STATIC_MAX_GROUPS (1 << 20)
#define LG_RANK_STATIC_MAX_TOP 4096
lg_status lg_rank_static(const float* score, int32_t n_groups, int32_t group_size, int32_t top_m,
                         int32_t* top_idx, float* top_score, int32_t* top_member, void* stream);

/* Tuning of the bucketed path; the autotuner sets it, the defaults work.
 * Ligands go to bucket (atom cluster, rotamer cluster): atom cluster c holds
 * atoms <= atom_bounds[c] (first match), rotamer cluster c bonds <=
 * rot_bounds[c]; the last cluster of each takes the rest.  A bucket is docked
 * by the kernel instance for ceil(atom bound / 64) atom slots per lane, with
 * waves_per_block[slots-1] wavefronts per block; its persistent grid is
 * grid_scale times the resident blocks of Eq. 1.  Work items are chunks of
 * restart_chunk restarts of one ligand.  Results do not depend on the tuning. */
typedef struct {
  int32_t n_atom_clusters;        /* 1..16 */
  int32_t atom_bounds[16];        /* increasing, each 1..LG_MAX_ATOMS */
  int32_t n_rot_clusters;         /* 1..32 */
  int32_t rot_bounds[32];         /* increasing, each 0..LG_MAX_TORSIONS */
  int32_t waves_per_block[4];     /* each 1, 2 or 4 */
  int32_t restart_chunk;          /* 1..LG_MAX_RESTARTS */
  int32_t grid_scale;             /* 1..64 */
  int32_t plain_waves_per_block;  /* 1, 2 or 4 */
  int32_t use_graph;              /* 1: capture once and replay as a HIP graph; 0: launch
                                     directly, with timing events around the bucket
                                     launches */
  int32_t lazy_clash;             /* 0: decide every torsion sample's clash test in the
                                     scoring pass (pruned pair list); 1: test only the
                                     winner and drop it while it clashes */
} lg_tuning;

lg_status lg_set_tuning(lg_pocket pocket, const lg_tuning* tuning);
lg_status lg_get_tuning(lg_pocket pocket, lg_tuning* tuning);

/* Autotuner of the bucketed path (the input-aware choices of Sec. 3 -- size
 * buckets and kernel shapes -- searched by measurement on the device).  Docks
 * the sample `ligands` with `params` (mode ignored: bucketed) repeatedly under
 * candidate tunings and keeps, by coordinate descent over `passes` passes, any
 * candidate at least 1 % faster: size buckets (one per kernel instance, with
 * or without rotamer clusters, or a single bucket), wavefronts per block of
 * each instance in use, restart chunk, persistent grid scale and the clash
 * test variant.  Times are the bucket launches of one call (events between
 * launches), best of two.  On success the handle keeps the best tuning (its
 * use_graph setting unchanged), *out receives it and *best_ms (optional) its
 * time (span of the bucket launches); on failure the handle's tuning is
 * restored.  Results never depend on
 * the tuning.  Synchronises `stream`; allocates its trial outputs. */
lg_status lg_autotune(lg_pocket pocket, const lg_ligands* ligands, const lg_dock_params* params, int32_t passes,
                      lg_tuning* out, float* best_ms, void* stream);

/* Per-bucket report of the last LG_BUCKETED call on a handle -- the MI355X
 * analog of the paper's Table 1 (registers and resident blocks per size class)
 * plus durations when the call ran with use_graph = 0 (events around every
 * launch).  Bucket launches run one after another on the caller's stream,
 * largest instance first, in both modes; span_ms covers all of them.
 * Fills up to `capacity` entries (NULL: none) and returns the number of bucket
 * launches, or a negative lg_status.  Synchronises the device to read ligand
 * counts and durations. */
typedef struct {
  int32_t bucket;            /* atom cluster * n_rot_clusters + rotamer cluster */
  int32_t atom_bound;        /* atoms <= atom_bound */
  int32_t rot_bound;         /* bonds <= rot_bound */
  int32_t slots;             /* atom slots per lane of the kernel instance */
  int32_t samples_per_lane;
  int32_t waves_per_block;
  int32_t vgprs;             /* architected VGPRs per lane of the instance */
  int32_t lds_bytes;         /* LDS per block */
  int32_t blocks_per_cu;     /* b of Eq. 1 */
  int32_t blocks;            /* persistent grid of the launch */
  int32_t ligands;           /* ligands in the bucket */
  float ms;                  /* launch duration, -1 if unknown */
  float span_ms;             /* first launch start to last launch end, -1 if unknown */
} lg_bucket_stat;

int32_t lg_bucket_stats(lg_pocket pocket, lg_bucket_stat* out, int32_t capacity);

/* Eq. 1 of the paper: ligands per bucket l = b * units * t / ws, with b the
 * resident blocks per compute unit of the class kernel, units the compute
 * units, t the threads per block and ws the wavefront size.  Host only. */
int64_t lg_bucket_size(int64_t blocks_per_unit, int64_t units, int64_t threads_per_block, int64_t wave_size);

/* Measurement aid for the ALU roofline of the kernels above: the sustained
 * rate, in lane-operations per second, of one non-packed VALU operation on the
 * handle's device -- eight independent chains per lane, eight wavefronts per
 * SIMD, `iters` iterations, timed with events on `stream` after one warm-up
 * launch.  kind: 0 v_fma_f32, 1 v_add_f32, 2 v_add_u32, 3 v_med3_f32,
 * 4 v_mad_i32_i24, 5 v_fma_f32 and v_add_u32 chains interleaved, 6 the
 * nearest-node index sequence of a scan sample (add, fma, med3, floor
 * conversion, shift-add, three-way add, and, conversion, add: ten operations).
 * Allocates and frees a small buffer; synchronises `stream`. */
lg_status lg_valu_probe(lg_pocket pocket, int32_t kind, int32_t iters, double* lane_ops_per_s, void* stream);

/* Cluster boundaries (Sec. 3): atom clusters at multiples of the wavefront
 * size (n_clusters-1 boundaries ws, 2ws, ..., the last cluster takes the
 * rest up to max_atoms); rotamer clusters split [0, max_rot] unevenly, finer at
 * low counts.  Writes inclusive upper bounds into bounds[n_clusters]; returns
 * the number written.  Host only. */
int32_t lg_atom_clusters(int32_t n_clusters, int32_t wave_size, int32_t max_atoms, int32_t* bounds);
int32_t lg_rotamer_clusters(int32_t n_clusters, int32_t max_rot, int32_t* bounds);

const char* lg_last_error(void);
int32_t lg_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LG_H_ */
