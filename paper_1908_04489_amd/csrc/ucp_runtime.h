// Host-side helpers shared by the solver API and the server (not public ABI).
#pragma once

#include <string>
#include <vector>

#include "ucp_internal.h"

namespace ucp {

// Launch-table kinds: one prefix array per kernel (and per search level).
enum : int {
  kKindMc0 = 0,                     // marginal-cost kernel, level l at kKindMc0 + l
  kKindSel0 = kKindMc0 + kMaxLevels,  // selection kernel, level l at kKindSel0 + l
  kKindU1p = kKindSel0 + kMaxLevels,
  kKindU1c,
  kKindJRows,
  kKindJRed,
  kKindPrior,
  kKindCopy,
  kKindFree,  // marginal-cost kernel on explicit candidates
  kKindFin,   // L_0 = f B for explicit candidates
  kKindGtab,  // offset table of the marginal-cost kernel
  kKindGt,    // moment table of the noise sums
  kKindU1s,   // culling data of the u1 sums (one unit per tile and per slice)
  kKindSelT0,  // selection kernel of instances with table_select, level l at kKindSelT0 + l
  kKinds = kKindSelT0 + kMaxLevels
};

extern thread_local std::string g_err;
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int check_problem(const ucp_problem* p);
int check_search(const ucp_search* s);
// relative tie band of the selection rule: the search's, or the default
double tie_band(const ucp_search* s);
int check_prec(int prec);
// UCP_FP64_GT needs a grid its moment table can serve (dy / s <= kGtStep)
int check_gt(const Inst& I);
Inst make_inst(const ucp_problem& p, const ucp_search* s, int prec, int cands_override);
size_t state_bytes(const Inst& I);
void carve_state(Inst& I, char*& base);
hipError_t clear_state(const Inst& I, hipStream_t st);
std::vector<int32_t> build_tables(const std::vector<Inst>& insts, const std::vector<char>& running);

hipError_t launch_v_from_u1(const Launch& L, hipStream_t st);

// The handle, for entry points defined outside ucp_api.cpp: its device, its
// workspace (grown to at least `bytes`; earlier contents are lost when it
// grows), and event pairs for timed launches (both null unless launches of
// `kind` are being timed; handle_harvest adds up the recorded pairs once the
// stream has been synchronised).
int handle_device(ucp_handle* h);
int handle_workspace(ucp_handle* h, size_t bytes, void** out);
hipError_t handle_events(ucp_handle* h, int kind, hipEvent_t* a, hipEvent_t* b);
bool handle_profiling(ucp_handle* h);
void handle_harvest(ucp_handle* h);

}  // namespace ucp
