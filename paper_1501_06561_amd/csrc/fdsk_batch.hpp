// Many independent sketches advanced together in lock-step rounds.
//
// The schedule of Algorithm 1 does not depend on the data (after a
// ReduceRank the surviving rows count as occupied, and a ReduceRank runs
// whenever all m rows are occupied), so the host knows in advance, for every
// sketch, which rows go into which buffer rows and when each ReduceRank runs.
// Round r holds at most one ingest and one ReduceRank per sketch; each stage
// of a round is one launch over all sketches active in it (the grid's last
// dimension indexes the task).  A sketch's ReduceRank kernels are the same
// device code as the single-sketch path.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fdsk_kernels.hpp"

namespace fdsk {

// Device workspace of one sketch (fixed for the life of the batch).
struct GroupSketch {
  double* C0;        // mp x ldc buffers (the rebuild writes the other one)
  double* C1;
  double* Gp;        // mp x mp Gram, lower tiles
  double* G;         // mp x mp Gram, symmetric
  double* W;         // mp x mp reflectors / tridiagonal
  double* V;         // mp x mp eigenvectors (column-major)
  double* Ut;        // mp x mp rebuild operator
  double* S1;        // mp x mp scratch (divide and conquer)
  double* S2;
  double* lam;       // mp
  double* rownorm;   // mp
  uint16_t* bh;      // bf16 halves of the buffer (npass > 0): hi then lo, rows64 x ldc each
  DevStats* st;
  int d, ldc, l, m, mp;
  int npass;         // Gram/rebuild products: 0 FP64, 1 BF16, 3 split-BF16 (compensated)
  RuleParams rp;
};

struct GroupIngest {      // f rows of src (leading dimension stride) into rows row0.. of C[cur]
  const void* src;
  int64_t stride;
  int sk, f, row0, cur;
};

struct GroupRR {          // a ReduceRank of sketch sk on C[cur]; rows [new0, new1) are new
  int sk, cur, new0, new1;
};

struct GroupSpan {        // rows [r0, r1) of C[cur] (zeroing, pending norms)
  int sk, cur, r0, r1;
};

// Launch shapes come from the host, which knows every task of the round.
hipError_t launch_group_ingest(const GroupSketch* sk, const GroupIngest* t, int nt, int max_f, int dt,
                               hipStream_t s);
// FP64 Gram for tasks with npass 0, then the symmetric mirror for every task.
hipError_t launch_group_gram(const GroupSketch* sk, const GroupRR* t, int nt, int max_mp, bool fp64,
                             hipStream_t s);
hipError_t launch_group_gram_lowp(const GroupSketch* sk, const GroupRR* t, int nt, int max_mp, int max_ldc,
                                  bool one, bool three, hipStream_t s);
hipError_t launch_group_rebuild_lowp(const GroupSketch* sk, const GroupRR* t, int nt, int max_ldc,
                                     int max_keep, bool one, bool three, hipStream_t s);
// The eigensolve of the tridiagonal route in its three stages (the head of
// the reduction only for buffers above the register capacity).
hipError_t launch_group_tridiag_head(const GroupSketch* sk, const GroupRR* t, int nt, int max_m,
                                     hipStream_t s);
hipError_t launch_group_tridiag(const GroupSketch* sk, const GroupRR* t, int nt, int max_m, hipStream_t s);
hipError_t launch_group_dc(const GroupSketch* sk, const GroupRR* t, int nt, hipStream_t s);
hipError_t launch_group_backtr(const GroupSketch* sk, const GroupRR* t, int nt, int max_m, hipStream_t s);
hipError_t launch_group_shrink(const GroupSketch* sk, const GroupRR* t, int nt, hipStream_t s);
// The FP64 rebuild for tasks with npass 0.
hipError_t launch_group_rebuild(const GroupSketch* sk, const GroupRR* t, int nt, int max_ldc, int max_keep,
                                hipStream_t s);
hipError_t launch_group_zero(const GroupSketch* sk, const GroupSpan* t, int nt, hipStream_t s);
hipError_t launch_group_pending(const GroupSketch* sk, const GroupSpan* t, int nt, hipStream_t s);

}  // namespace fdsk
