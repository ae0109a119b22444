// Host-side checks of the C ABI's arguments and the host-only calls; plain C++.
#include "host_checks.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>

namespace lghost {

// The last error message of the calling thread; a fixed buffer, so recording
// an error never allocates (it may be the report of a failed allocation).
thread_local char g_err[512];

lg_status fail(lg_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return s;
}

// Debug and test controls read from the environment at every call:
// LG_WORKSPACE_LIMIT (bytes) caps the docking workspace and stream buffers;
// LG_FAULT_AFTER_CHUNKS=k makes lg_dock_stream stop with LG_ERR_DEVICE after
// k chunks of a call (the finished chunks' outputs and manifest entries kept).
long long env_ll(const char* name, long long dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  char* end = nullptr;
  const long long x = std::strtoll(v, &end, 10);
  return (end && *end == 0 && x >= 0) ? x : dflt;
}

size_t workspace_limit() { return (size_t)env_ll("LG_WORKSPACE_LIMIT", (long long)(SIZE_MAX >> 1)); }

lg_status check_ligands(const lg_ligands* L, bool need_tors) {
  if (!L) return fail(LG_ERR_INVALID_ARG, "ligands is NULL");
  if (L->n < 0) return fail(LG_ERR_INVALID_ARG, "n = %d < 0", L->n);
  if (L->n == 0) return LG_OK;
  if (!L->atom_offset || !L->tors_offset || !L->x || !L->y || !L->z || !L->ref_point)
    return fail(LG_ERR_INVALID_ARG, "a required ligand array is NULL");
  if (need_tors && (!L->frag_mask || (L->total_torsions > 0 && (!L->tors_atoms || !L->inv_bond_len))))
    return fail(LG_ERR_INVALID_ARG, "a required ligand array is NULL");
  if (L->total_atoms < L->n || L->total_torsions < 0) return fail(LG_ERR_INVALID_ARG, "bad total sizes");
  if (L->total_atoms > (1 << 30) - 256)
    return fail(LG_ERR_LIMIT, "total_atoms %d above 2^30 - 256 (32-bit byte offsets)", L->total_atoms);
  if (L->atom_offset_host) {
    for (int i = 0; i < L->n; ++i) {
      const long long N = (long long)L->atom_offset_host[i + 1] - L->atom_offset_host[i];
      if (N < 1 || N > LG_MAX_ATOMS) return fail(LG_ERR_LIMIT, "ligand %d has %lld atoms (1..%d)", i, N, LG_MAX_ATOMS);
    }
    if (L->atom_offset_host[0] != 0 || L->atom_offset_host[L->n] != L->total_atoms)
      return fail(LG_ERR_INVALID_ARG, "atom_offset does not span [0, total_atoms)");
  }
  if (L->tors_offset_host) {
    for (int i = 0; i < L->n; ++i) {
      const long long K = (long long)L->tors_offset_host[i + 1] - L->tors_offset_host[i];
      if (K < 0 || K > LG_MAX_TORSIONS) return fail(LG_ERR_LIMIT, "ligand %d has %lld bonds (0..%d)", i, K, LG_MAX_TORSIONS);
    }
    if (L->tors_offset_host[0] != 0 || L->tors_offset_host[L->n] != L->total_torsions)
      return fail(LG_ERR_INVALID_ARG, "tors_offset does not span [0, total_torsions)");
  }
  if (L->tors_atoms_host) {
    if (!L->atom_offset_host || !L->tors_offset_host)
      return fail(LG_ERR_INVALID_ARG, "tors_atoms_host needs atom_offset_host and tors_offset_host");
    for (int i = 0; i < L->n; ++i) {
      const long long N = (long long)L->atom_offset_host[i + 1] - L->atom_offset_host[i];
      for (int k = L->tors_offset_host[i]; k < L->tors_offset_host[i + 1]; ++k) {
        const int a = L->tors_atoms_host[2 * k], b = L->tors_atoms_host[2 * k + 1];
        if (a < 0 || a >= N || b < 0 || b >= N || a == b)
          return fail(LG_ERR_INVALID_ARG, "ligand %d: bond %d has atom ids (%d, %d), need two distinct ids in 0..%lld",
                      i, k, a, b, N - 1);
      }
    }
  }
  return LG_OK;
}

// Largest atom and bond count of a batch whose three host copies were checked by
// check_ligands; -1 when a copy is missing (the device check then supplies them).
void host_maxima(const lg_ligands* L, int* max_atoms, int* max_tors) {
  *max_atoms = *max_tors = -1;
  if (!L || L->n < 1 || !L->atom_offset_host || !L->tors_offset_host || !L->tors_atoms_host) return;
  int ma = 0, mt = 0;
  for (int i = 0; i < L->n; ++i) {
    ma = std::max(ma, L->atom_offset_host[i + 1] - L->atom_offset_host[i]);
    mt = std::max(mt, L->tors_offset_host[i + 1] - L->tors_offset_host[i]);
  }
  *max_atoms = ma;
  *max_tors = mt;
}

// Host-side validation of a host-resident library (the device check's rules):
// offsets from 0, non-decreasing, totals; 1..LG_MAX_ATOMS atoms and
// 0..LG_MAX_TORSIONS bonds per ligand; bond atoms are two distinct local ids.
lg_status check_host_ligands(const lg_host_ligands* H) {
  if (!H) return fail(LG_ERR_INVALID_ARG, "ligands is NULL");
  if (H->n < 0 || H->total_atoms < 0 || H->total_torsions < 0) return fail(LG_ERR_INVALID_ARG, "negative sizes");
  if (!H->atom_offset || !H->tors_offset) return fail(LG_ERR_INVALID_ARG, "offsets are required");
  if (H->n > 0 && (!H->x || !H->y || !H->z || !H->frag_mask || !H->ref_point))
    return fail(LG_ERR_INVALID_ARG, "x, y, z, frag_mask and ref_point are required");
  if (H->total_torsions > 0 && (!H->tors_atoms || !H->inv_bond_len))
    return fail(LG_ERR_INVALID_ARG, "tors_atoms and inv_bond_len are required");
  if (H->atom_offset[0] != 0 || H->tors_offset[0] != 0 || H->atom_offset[H->n] != H->total_atoms ||
      H->tors_offset[H->n] != H->total_torsions)
    return fail(LG_ERR_INVALID_ARG, "offsets must start at 0 and end at the totals");
  // every offset first: only a fully checked (non-decreasing, in-range) list may
  // index the bond array
  for (int i = 0; i < H->n; ++i) {
    const long long N = (long long)H->atom_offset[i + 1] - H->atom_offset[i];
    const long long K = (long long)H->tors_offset[i + 1] - H->tors_offset[i];
    if (N < 1 || N > LG_MAX_ATOMS) return fail(LG_ERR_LIMIT, "ligand %d has %lld atoms, allowed 1..%d", i, N, LG_MAX_ATOMS);
    if (K < 0 || K > LG_MAX_TORSIONS) return fail(LG_ERR_LIMIT, "ligand %d has %lld bonds, allowed 0..%d", i, K, LG_MAX_TORSIONS);
  }
  for (int i = 0; i < H->n; ++i) {
    const long long N = (long long)H->atom_offset[i + 1] - H->atom_offset[i];
    for (int k = H->tors_offset[i]; k < H->tors_offset[i + 1]; ++k)
      if (H->tors_atoms[2 * k] < 0 || H->tors_atoms[2 * k] >= N || H->tors_atoms[2 * k + 1] < 0 ||
          H->tors_atoms[2 * k + 1] >= N || H->tors_atoms[2 * k] == H->tors_atoms[2 * k + 1])
        return fail(LG_ERR_INVALID_ARG, "ligand %d: bond %d needs two distinct atom ids in 0..%lld", i, k, N - 1);
  }
  return LG_OK;
}

lg_status check_tuning(const lg_tuning* t) {
  if (t->n_atom_clusters < 1 || t->n_atom_clusters > 16 || t->n_rot_clusters < 1 || t->n_rot_clusters > 32)
    return fail(LG_ERR_INVALID_ARG, "cluster counts out of range");
  for (int c = 0; c < t->n_atom_clusters; ++c)
    if (t->atom_bounds[c] < 1 || t->atom_bounds[c] > LG_MAX_ATOMS || (c && t->atom_bounds[c] <= t->atom_bounds[c - 1]))
      return fail(LG_ERR_INVALID_ARG, "atom bounds must increase within 1..%d", LG_MAX_ATOMS);
  for (int c = 0; c < t->n_rot_clusters; ++c)
    if (t->rot_bounds[c] < 0 || t->rot_bounds[c] > LG_MAX_TORSIONS || (c && t->rot_bounds[c] <= t->rot_bounds[c - 1]))
      return fail(LG_ERR_INVALID_ARG, "rotamer bounds must increase within 0..%d", LG_MAX_TORSIONS);
  for (int i = 0; i < 4; ++i)
    if (t->waves_per_block[i] != 1 && t->waves_per_block[i] != 2 && t->waves_per_block[i] != 4)
      return fail(LG_ERR_INVALID_ARG, "waves_per_block must be 1, 2 or 4");
  if (t->plain_waves_per_block != 1 && t->plain_waves_per_block != 2 && t->plain_waves_per_block != 4)
    return fail(LG_ERR_INVALID_ARG, "plain_waves_per_block must be 1, 2 or 4");
  if (t->restart_chunk < 1 || t->restart_chunk > LG_MAX_RESTARTS || t->grid_scale < 1 || t->grid_scale > 64)
    return fail(LG_ERR_INVALID_ARG, "restart_chunk in 1..%d and grid_scale in 1..64", LG_MAX_RESTARTS);
  if (t->use_graph != 0 && t->use_graph != 1) return fail(LG_ERR_INVALID_ARG, "use_graph must be 0 or 1");
  if (t->lazy_clash != 0 && t->lazy_clash != 1) return fail(LG_ERR_INVALID_ARG, "lazy_clash must be 0 or 1");
  return LG_OK;
}

void copy_slice(size_t bytes, int slices, int s, size_t* b0, size_t* b1) {
  const size_t per = bytes / (size_t)slices;
  *b0 = std::min(bytes, (per * (size_t)s) & ~(size_t)4095);
  *b1 = s == slices - 1 ? bytes : std::min(bytes, (per * (size_t)(s + 1)) & ~(size_t)4095);
}

}  // namespace lghost

using lghost::g_err;

extern "C" {

const char* lg_last_error(void) { return g_err; }

int32_t lg_version(void) { return 1; }

int64_t lg_bucket_size(int64_t blocks_per_unit, int64_t units, int64_t threads_per_block, int64_t wave_size) {
  if (blocks_per_unit < 0 || units < 0 || threads_per_block <= 0 || wave_size <= 0) return -1;
  return blocks_per_unit * units * threads_per_block / wave_size;
}

int32_t lg_atom_clusters(int32_t n_clusters, int32_t wave_size, int32_t max_atoms, int32_t* bounds) {
  if (n_clusters < 1 || wave_size < 1 || max_atoms < 1 || !bounds) return 0;
  int c = 0;
  for (; c < n_clusters - 1 && (c + 1) * wave_size < max_atoms; ++c) bounds[c] = (c + 1) * wave_size;
  bounds[c++] = max_atoms;
  return c;
}

int32_t lg_rotamer_clusters(int32_t n_clusters, int32_t max_rot, int32_t* bounds) {
  if (n_clusters < 1 || max_rot < 0 || !bounds) return 0;
  int c = 0, prev = -1;
  for (int i = 0; i < n_clusters - 1; ++i) {
    double f = (double)(i + 1) / n_clusters;
    int b = (int)std::lround(max_rot * f * f);
    b = std::max(b, prev + 1);
    if (b >= max_rot) break;
    bounds[c++] = b;
    prev = b;
  }
  bounds[c++] = max_rot;
  return c;
}

}  // extern "C"
