// Internal declarations shared by the engine's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

// Device copy of a compiled gate list.
struct GateTable {
  const int* bond;
  const int* kind;
  const zd* pre;     // [G][16]
  const zd* post;    // [G][16]
  const int* param;
  const double* coeff;
  int G;
};

// Accumulated per-call statistics (device).
struct GateStats {
  double disc_sum;
  double disc_max;
  int truncated;
  int max_sweeps;
  int noconv;
  int degenerate_cuts;
  int max_bond;
  int gates;
  int degen_grad;    // degenerate pairs that carried a cotangent (backward)
  int pad;
};

// Workspace of one gate update.
struct GateWork {
  zd* C;          // [ncap][ldc] column-major, unweighted C
  zd* A;          // [ncap][ldc] weighted C, orthogonalised in place
  zd* V;          // [ncap][ldv]
  double* sv;     // [ncap]
  int* perm;      // [ncap]
  int* gmeta;     // [4]
  double* gdmeta; // [4]
  int* rotflag;   // [128]
  GateStats* stats;
  int ldc, ldv, ncap;
  double eps, tol;
  int dmax, max_sweeps;
};

struct SvdArgs {
  zd* A;
  int lda;
  zd* V;
  int ldv;
  int* dims;
  int bond;
  double* sv;
  int* perm;
  int* gmeta;
  double* gdmeta;
  int* rotflag;
  double* lam_out;
  GateStats* stats;
  double eps;
  int dmax;
  double tol;
  int max_sweeps;
};

int svd_width(int dcap);
hipError_t launch_gate(const MpsView& st, const GateTable& gt, int g, int bond, const double* theta,
                       GateWork& w, hipStream_t stream);
hipError_t svd_set_attributes(int dcap, size_t shm);

// ----------------------------------------------------------------------------
// Pauli sweeps
// ----------------------------------------------------------------------------
// One transfer job at a site: L_out = sum_i o_i (B^{i^x})^dagger L_in B^i.
struct SweepJob {
  int in_slot;    // -1: start from the identity environment of this site
  int out_slot;
  int xb;         // bit flip of the site operator
  int pad;
  zd o0, o1;      // O[i^x, i] = o_i
};

struct SweepBuffers {
  zd* Lid;        // [N+1][dcap][dcap] identity left environments
  zd* Rid;        // [N+1][dcap][dcap] identity right environments
  zd* Lslots;     // [chunk][dcap][dcap]
  zd* Y;          // [chunk][dcap][2 dcap] stage-1 products
  zd* Yid;        // [2 dcap][dcap] scratch for identity environments
  zd* termval;    // [K] unnormalised <P_k>
  double* energy; // [4]: E, Im E, Z, c0 sum
  int chunk;
};

hipError_t launch_identity_envs(const MpsView& st, SweepBuffers& sb, hipStream_t stream);
hipError_t launch_transfer(const MpsView& st, SweepBuffers& sb, int n, const SweepJob* jobs, int njobs,
                           hipStream_t stream);
hipError_t launch_finalize(const MpsView& st, SweepBuffers& sb, int n, const int* slots, const int* terms,
                           int nfin, hipStream_t stream);
hipError_t launch_energy_sum(const MpsView& st, SweepBuffers& sb, const double* coeff, int64_t K, double c0,
                             hipStream_t stream);

__global__ void k_init_product(MpsView st, const uint8_t* occ);
