// pipeline.hip -- host-side verifier state of pipelined LSD (Alg. 2).
//
// The pipelined algorithm submits every draft step for verification as soon
// as it is drafted and lets target results return in any order.  The main
// loop keeps three buffers keyed by the step id (unique, ascending):
//   EP  eligible pending: submitted, not returned, not flushed;
//   CV  conditionally verified: returned, with every predecessor not yet
//       known to be accepted;
//   V   verified: the output trajectory, in id order.
// A return of a flushed step is ignored.  A return of a step in EP moves it
// to CV; if it was rejected, every later step is flushed from EP and CV and
// the draft rolls back to the rejected step's target state.  Then the
// smallest CV id moves to V while it precedes every EP id.  The step states
// themselves stay with the caller, who keeps them by id.
#include <algorithm>
#include <set>
#include <vector>

#include "lsd.h"

lsd_status lsd_record_error(lsd_status s, const char* msg);  // lsd_api.hip

struct lsd_pipeline {
  int64_t next_id = 1;    // id 0 is the initial state, verified from the start
  std::set<int64_t> ep;   // eligible pending
  std::set<int64_t> cv;   // conditionally verified
  int64_t n_verified = 1;
  std::vector<int64_t> fresh;  // ids appended to V since the last take
};

extern "C" {

lsd_status lsd_pipeline_create(lsd_pipeline** out) {
  if (!out) return lsd_record_error(LSD_ERR_INVALID_ARG, "null argument");
  *out = new lsd_pipeline();
  return LSD_OK;
}

lsd_status lsd_pipeline_destroy(lsd_pipeline* p) {
  delete p;
  return LSD_OK;
}

lsd_status lsd_pipeline_submit(lsd_pipeline* p, int64_t* id) {
  if (!p || !id) return lsd_record_error(LSD_ERR_INVALID_ARG, "null argument");
  *id = p->next_id++;
  p->ep.insert(*id);
  return LSD_OK;
}

lsd_status lsd_pipeline_return(lsd_pipeline* p, int64_t id, int32_t accepted, int32_t* ignored,
                               int32_t* rollback) {
  if (!p || !ignored || !rollback) return lsd_record_error(LSD_ERR_INVALID_ARG, "null argument");
  if (id < 1 || id >= p->next_id)
    return lsd_record_error(LSD_ERR_INVALID_ARG, "step id was never submitted");
  *ignored = 0;
  *rollback = 0;
  auto it = p->ep.find(id);
  if (it == p->ep.end()) {
    *ignored = 1;  // flushed by an earlier rejection (or returned twice)
    return LSD_OK;
  }
  p->ep.erase(it);
  p->cv.insert(id);
  if (!accepted) {
    p->ep.erase(p->ep.upper_bound(id), p->ep.end());
    p->cv.erase(p->cv.upper_bound(id), p->cv.end());
    *rollback = 1;
  }
  while (!p->cv.empty() && (p->ep.empty() || *p->cv.begin() < *p->ep.begin())) {
    p->fresh.push_back(*p->cv.begin());
    p->cv.erase(p->cv.begin());
    ++p->n_verified;
  }
  return LSD_OK;
}

lsd_status lsd_pipeline_take_verified(lsd_pipeline* p, int64_t* ids, int32_t cap, int32_t* n) {
  if (!p || !n || cap < 0 || (cap > 0 && !ids))
    return lsd_record_error(LSD_ERR_INVALID_ARG, "bad argument");
  const int32_t k = (int32_t)std::min<size_t>((size_t)cap, p->fresh.size());
  std::copy(p->fresh.begin(), p->fresh.begin() + k, ids);
  p->fresh.erase(p->fresh.begin(), p->fresh.begin() + k);
  *n = k;
  return LSD_OK;
}

lsd_status lsd_pipeline_counts(const lsd_pipeline* p, int64_t* out) {
  if (!p || !out) return lsd_record_error(LSD_ERR_INVALID_ARG, "null argument");
  out[0] = (int64_t)p->ep.size();
  out[1] = (int64_t)p->cv.size();
  out[2] = p->n_verified;
  return LSD_OK;
}

}  // extern "C"
