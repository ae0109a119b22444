// Host-side checks of the C ABI's arguments, in plain C++ (no device code), so
// that they also build with the host compiler's address and undefined-behaviour
// sanitizers: ligand batches (device batches with optional host copies, and
// host-resident libraries), tunings, and the host-only calls (Eq. 1, cluster
// boundaries, the last error message).  The check functions report failures
// through fail(), which records the message lg_last_error() returns.
#pragma once
#include <cstddef>
#include <exception>
#include <new>

#include "lg.h"

namespace lghost {

lg_status fail(lg_status s, const char* fmt, ...);

// Environment controls read at every call (a non-negative integer, else dflt).
long long env_ll(const char* name, long long dflt);
size_t workspace_limit();

// A device batch: sizes, limits and (when host copies are given) offsets and bond ids.
lg_status check_ligands(const lg_ligands* L, bool need_tors);
// Largest atom and bond count from the three host copies, or -1 when one is missing.
void host_maxima(const lg_ligands* L, int* max_atoms, int* max_tors);
// A host-resident library (lg_dock_stream): the device check's rules, on the host.
lg_status check_host_ligands(const lg_host_ligands* H);
lg_status check_tuning(const lg_tuning* t);

// Byte range [*b0, *b1) of slice s of `slices` page-aligned slices of a
// `bytes`-long copy (the last slice ends at `bytes`; the slices tile the range
// in order, some possibly empty).
void copy_slice(size_t bytes, int slices, int s, size_t* b0, size_t* b1);

// No C++ exception crosses the C ABI: a host allocation that fails inside a
// call (std::bad_alloc) becomes LG_ERR_OUT_OF_MEMORY, anything else thrown
// LG_ERR_DEVICE, with the message recorded.  A guarded body that throws must
// leave no device memory that its pocket does not own and free nothing the
// device may still be using.
template <class F>
auto guarded(F&& f) noexcept -> decltype(f()) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(LG_ERR_OUT_OF_MEMORY, "host memory could not be allocated");
  } catch (const std::exception& e) {
    return fail(LG_ERR_DEVICE, "host-side failure: %s", e.what());
  } catch (...) {
    return fail(LG_ERR_DEVICE, "host-side failure");
  }
}

}  // namespace lghost
