// Host-side helpers shared between the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/sem.h"

namespace sem {

// The handle's stream and the node count of its finest level (false for a
// null handle).
bool handle_top(sem_handle h, hipStream_t *stream, long *nodes);
// Records msg as the handle's last error.
void handle_error(sem_handle h, const char *msg);
// Resolves the allocation-free entry points' device array on the current
// device (once per device); false when the runtime call fails.
bool noalloc_prepare();

// Host description of the subdomain types along one direction.
struct DirFdm {
  int ntypes = 0;
  std::vector<int> type_of;       // per element
  std::vector<double> S, ST, SW, lam;  // per type m*m (S, S^T, diag(w) S), m
  std::vector<double> wts;        // per element m
};

// Subdomain types, factors and weights along one direction (Section 3.1):
// br = n + 1 element breaks, windows of n_o layers, weight function wf
// (alpha: optional width scale per grid line; unweighted: unit weights, the
// per-element or multiplicative cases).
DirFdm build_direction(const std::vector<double> &br, int p, int n_o, int periodic, int wf,
                       const double *alpha, bool unweighted = false);

}  // namespace sem
