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

#include <algorithm>

#include "fdsk_kernels.hpp"

namespace fdsk {

// Device workspace of one sketch (fixed for the life of the batch).
struct GroupSketch {
  double* C0;        // mp x ldc buffers (the rebuild writes the other one)
  double* C1;
  double* Gp;        // gp_parts(ldc) x mp x mp Gram partials, lower tiles
  double* G;         // mp x mp Gram, symmetric
  double* W;         // mp x mp reflectors / tridiagonal
  double* V;         // mp x mp eigenvectors (column-major)
  double* Ut;        // mp x mp rebuild operator
  double* S1;        // mp x mp scratch (divide and conquer)
  double* S2;
  double* lam;       // mp
  double* rownorm;   // mp
  uint16_t* bh0;     // bf16 halves of C0 / C1 (npass > 0): hi then lo, rows64 x ldc each,
  uint16_t* bh1;     // written by the ingest and the rebuild beside the FP64 rows
  uint16_t* uh;      // Ut's split-BF16 halves (npass > 0): hi rows then lo rows, mp x mp each
  DevStats* st;
  int d, ldc, l, m, mp;
  int npass;         // Gram/rebuild products: 0 FP64, 1 BF16, 3 split-BF16 (compensated)
  int kchunk;        // Gram K slice length (see task_kchunk), tuned per size class
  RuleParams rp;
};

// w64: write the FP64 rows too.  A split-BF16 sketch's products read only
// the bf16 halves, so its FP64 rows are needed only where finalize may copy
// them out: rows that no later ReduceRank of the same append call consumes.
// The host knows which those are (the schedule does not depend on the
// data); FP64 sketches always write them.
struct GroupIngest {      // f rows of src (leading dimension stride) into rows row0.. of C[cur]
  const void* src;
  int64_t stride;
  int sk, f, row0, cur, w64, pad;
};

struct GroupRR {          // a ReduceRank of sketch sk on C[cur]; rows [new0, new1) are new
  int sk, cur, new0, new1, w64;   // w64: the rebuild writes its FP64 rows
};

struct GroupSpan {        // rows [r0, r1) of C[cur] (zeroing, pending norms)
  int sk, cur, r0, r1;
};

// Launch shapes come from the host, which knows every task of the round.
hipError_t launch_group_ingest(const GroupSketch* sk, const GroupIngest* t, int nt, int max_f, int dt,
                               hipStream_t s);
// Gram products split along K: a task's row length is cut into slices of
// task_kchunk(kc, ldc) columns, one partial per slice in the task's Gp,
// which holds gp_parts(ldc) partials.  kc is the sketch's own slice length
// (GroupSketch::kchunk: 0 = one slice, else 256, 512 or 1024), raised where
// needed so that no task has more than kGpParts slices; it depends on the
// sketch alone, so results do not depend on how tasks are grouped.
constexpr int kGpParts = 8;
inline int gp_parts(int ldc) { return std::max(1, std::min(kGpParts, (ldc + 255) / 256)); }
__host__ __device__ inline int task_kchunk(int kc, int ldc) {
  if (kc <= 0) return ldc;
  const int lo = ((ldc + kGpParts - 1) / kGpParts + 63) / 64 * 64;
  return kc > lo ? kc : lo;
}
// FP64 Gram for tasks with npass 0, then the sum of every task's partials
// and the symmetric mirror.  ks: the largest slice count of the tasks (the
// grid's K dimension).  kc >= 0 replaces every task's own kchunk (the
// tuner's candidates); -1 uses them.
hipError_t launch_group_gram(const GroupSketch* sk, const GroupRR* t, int nt, int max_mp, bool fp64, int ks,
                             int kc, hipStream_t s);
hipError_t launch_group_gram_lowp(const GroupSketch* sk, const GroupRR* t, int nt, int max_mp, int max_ldc,
                                  bool one, bool three, int ks, int kc, hipStream_t s);
// Rebuilds with rt (32 or 64) rows per workgroup.
hipError_t launch_group_rebuild_lowp(const GroupSketch* sk, const GroupRR* t, int nt, int max_ldc,
                                     int max_keep, bool one, bool three, int rt, hipStream_t s);
// The eigensolve of the tridiagonal route in its three stages (the head of
// the reduction only for buffers above the register capacity).
hipError_t launch_group_tridiag_head(const GroupSketch* sk, const GroupRR* t, int nt, int max_m,
                                     hipStream_t s);
hipError_t launch_group_tridiag(const GroupSketch* sk, const GroupRR* t, int nt, int max_m, hipStream_t s);
hipError_t launch_group_dc(const GroupSketch* sk, const GroupRR* t, int nt, int max_m, hipStream_t s);
// max_c: the most eigenvectors any task wants (min(m, l)).
hipError_t launch_group_backtr(const GroupSketch* sk, const GroupRR* t, int nt, int max_m, int max_c,
                               hipStream_t s);
hipError_t launch_group_shrink(const GroupSketch* sk, const GroupRR* t, int nt, hipStream_t s);
// The FP64 rebuild for tasks with npass 0.
hipError_t launch_group_rebuild(const GroupSketch* sk, const GroupRR* t, int nt, int max_ldc, int max_keep,
                                int rt, hipStream_t s);
hipError_t launch_group_zero(const GroupSketch* sk, const GroupSpan* t, int nt, hipStream_t s);
hipError_t launch_group_pending(const GroupSketch* sk, const GroupSpan* t, int nt, hipStream_t s);

}  // namespace fdsk
