// Launch interface between the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "hyb.h"
#include "hyb_internal.h"

namespace hyb {

// One entry per workgroup of a batched launch: which run it serves, its
// block index inside that run and how many blocks the run has.
struct BlockMap { int run, lb, nb, pad; };

struct Plan {
  BlockMap* map = nullptr;   // device array [nb]
  int nb = 0;
};

// Everything one step needs: the run descriptors and one plan per phase.
struct LaunchSet {
  const RunDesc* runs = nullptr;   // device array [nruns]
  int nruns = 0;
  Plan zero, inject, particle, gather, grid, cells, fin, adv;
  Plan scan, scan1;   // tile-count scan: one block per kScanTile tiles; one block per run
  bool sort = false;                                  // some run sorts its particles
  bool delta = false;                                 // some run has delta rays
  bool urban = false;                                 // some run has the Urban-type scatter
  bool compound = false;                              // some run's solid has several elements
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;   // optional timing of the particle kernel
  // optional streams (default priority) and the events that fork the field
  // sub-cycles and the heating onto them beside the sort, and join them back
  hipStream_t side = nullptr, side2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_join2 = nullptr;
};

void launch_step(const LaunchSet& L, hipStream_t s, int precision, int max_sub);
void launch_kinetic(const RunDesc* runs, int run, int nblocks, hipStream_t s, int precision);
// the energy-partition model at n scan points (device arrays; out 6 n doubles)
void launch_model(const hyb_model& m, const double* I0, const double* Z, long long n, double* out,
                  hipStream_t s);

}  // namespace hyb
