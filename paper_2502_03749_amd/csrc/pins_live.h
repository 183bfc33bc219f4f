// pins_live.h -- live batch: the engine of the serving runtime (internal).
//
// A live batch holds up to max_slots problems on one HIP stream and advances
// all of them one outer iteration of Alg. 2 per round.  Problems are admitted
// between rounds (each starts its own outer loop at k = 0 while the others
// continue theirs) and leave when their K outer iterations are done, so
// requests join and leave a running batch at outer-iteration boundaries.
// Each problem's workspace and input/output staging is carved from one device
// arena (first fit); the per-instance control blocks keep every problem's own
// outer counter and tolerances, so a problem's arithmetic does not depend on
// which others share its rounds.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "pins.h"

namespace pins {

struct LiveBatch;

struct LiveDone {
    int64_t id;      // the caller's id of the problem
    int rc;          // its status (pins_status)
    pins_result res; // scalars (alpha/beta/X pointers unset)
};

// A live batch on `device` with parameters p (implicit shift; Hessian products
// sparsified or matrix-free throughout, hvp 0 or 1), room for max_slots
// problems and an arena of arena_bytes.  Throws nothing; nullptr and *err on
// failure.
LiveBatch* live_create(int device, const pins_params& p, int max_slots, size_t arena_bytes, std::string* err);
void live_destroy(LiveBatch* B);
// problems in the batch, and whether they are GRID problems (a batch holds one family)
int live_count(const LiveBatch* B);
bool live_grid(const LiveBatch* B);
// arena bytes a problem needs (its workspace plus input and output staging)
size_t live_bytes(const LiveBatch* B, const pins_problem& prob);
// Admit a problem given by HOST pointers (read during the call; alpha_out and
// beta_out, HOST arrays of m and n doubles, are written when it completes).
// Returns false when no slot or arena room is free, or its family differs.
bool live_admit(LiveBatch* B, int64_t id, const pins_problem& prob, double* alpha_out, double* beta_out);
// One round: set-up of the newly admitted problems, one outer iteration of
// every problem, outputs of those that finished.  Completed problems (and
// those rejected at set-up) are appended to done and leave the batch.
// Returns PINS_OK, or a negative status after a device failure (every problem
// of the batch is then completed with it).
int live_round(LiveBatch* B, std::vector<LiveDone>& done, std::string* err);

}  // namespace pins
