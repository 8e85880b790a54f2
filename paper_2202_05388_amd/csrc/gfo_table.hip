// Grouped greedy steps of many resident jobs (the served form): one launch per
// move steps every job of a table, instead of one launch per job and move.
// Small jobs are latency bound (a 24 x 24 job's move is a few microseconds of
// device work), so their launches, not the device, bound a served burst.
#include "gfo_internal.hpp"

#include <vector>

namespace gfo {

constexpr int kTableMaxJobs = 64;   // the per-move "flushed" flags travel as one 64-bit word

// Every job of a grouped call: valid, deferred, served by the one-kernel loop,
// and alike in what selects the kernel instance (storage type, term batch,
// summaries per lane).
static int check_group(const gfo_problem* probs, const gfo_state* states, int n_jobs,
                       std::vector<Geo>* geos, std::vector<Layout>* lays) {
  if (!probs || !states || n_jobs < 1 || n_jobs > kTableMaxJobs) return GFO_EINVAL;
  geos->resize(n_jobs);
  lays->resize(n_jobs);
  for (int i = 0; i < n_jobs; ++i) {
    int rc = validate_job(&probs[i], &states[i], &(*lays)[i]);
    if (rc) return rc;
    if (states[i].delay <= 0) return GFO_EINVAL;
    (*geos)[i] = make_geo(&probs[i], &states[i]);
    if (!one_kernel_loop((*geos)[i])) return GFO_EINVAL;
    if (i > 0) {
      if ((*geos)[i].dtype != (*geos)[0].dtype) return GFO_EINVAL;
      if ((states[i].delay <= 64) != (states[0].delay <= 64)) return GFO_EINVAL;
      if (move_small_grid((*geos)[i]) != move_small_grid((*geos)[0])) return GFO_EINVAL;
    }
  }
  return GFO_OK;
}

}  // namespace gfo

using namespace gfo;

extern "C" size_t gfo_job_table_bytes(int32_t n_jobs) {
  if (n_jobs < 1 || n_jobs > kTableMaxJobs) return 0;
  return (size_t)n_jobs * sizeof(JobEntry);
}

extern "C" int gfo_job_table_build(const gfo_problem* probs, const gfo_state* states,
                                   int32_t n_jobs, const uint32_t* h_cand_masks,
                                   const double* h_taus, void* d_table, size_t table_bytes,
                                   hipStream_t stream) {
  discard_stale_hip();
  std::vector<Geo> geos;
  std::vector<Layout> lays;
  int rc = check_group(probs, states, n_jobs, &geos, &lays);
  if (rc) return rc;
  if (!h_cand_masks || !h_taus || !d_table || ((uintptr_t)d_table & 255) != 0) return GFO_EINVAL;
  if (table_bytes < gfo_job_table_bytes(n_jobs)) return GFO_ENOSPC;
  std::vector<JobEntry> tab(n_jobs);
  for (int i = 0; i < n_jobs; ++i) {
    const uint32_t mask = h_cand_masks[i] & ((1u << probs[i].n_eps) - 1u);
    const double tau = h_taus[i];
    if (mask == 0 || !(tau >= 0.0) || !(tau < 1.0)) return GFO_EINVAL;
    tab[i] = make_job_entry(geos[i], &states[i], lays[i], mask, tau);
  }
  if (note_hip(hipMemcpyAsync(d_table, tab.data(), tab.size() * sizeof(JobEntry),
                              hipMemcpyHostToDevice, stream)) != hipSuccess ||
      note_hip(hipStreamSynchronize(stream)) != hipSuccess)
    return GFO_EHIP;
  return GFO_OK;
}

extern "C" int gfo_greedy_steps_table(const gfo_problem* probs, gfo_state* states, int32_t n_jobs,
                                      int32_t n_steps, const void* d_table, hipStream_t stream) {
  discard_stale_hip();
  std::vector<Geo> geos;
  std::vector<Layout> lays;
  int rc = check_group(probs, states, n_jobs, &geos, &lays);
  if (rc) return rc;
  if (!d_table || n_steps < 0) return GFO_EINVAL;
  if (n_steps == 0) return GFO_OK;
  const JobEntry* tab = (const JobEntry*)d_table;
  const Geo& g0 = geos[0];
  const bool c64 = g0.dtype == GFO_C64;
  const bool small = move_small_grid(g0);
  const int batch = states[0].delay <= 64 ? 16 : 32;
  int wg_score = 0, wg_move = 0, wg_finish = 0;
  for (int i = 0; i < n_jobs; ++i) {
    const JobEntry je = make_job_entry(geos[i], &states[i], lays[i], 0, 0.0);
    wg_score = je.n_score_wg > wg_score ? je.n_score_wg : wg_score;
    wg_move = je.n_move_wg > wg_move ? je.n_move_wg : wg_move;
    wg_finish = je.n_finish_wg > wg_finish ? je.n_finish_wg : wg_finish;
  }
  // the call's first scores, for every job
  if ((c64 ? launch_table_scores<float2>(tab, n_jobs, wg_score, stream)
           : launch_table_scores<double2>(tab, n_jobs, wg_score, stream)) != hipSuccess)
    return GFO_EHIP;
  for (int t = 0; t < n_steps; ++t) {
    // a job whose term buffer is full is flushed before its move, as in its own
    // call (the previous move's pivot values reach memory first)
    uint64_t flushed = 0;
    for (int i = 0; i < n_jobs; ++i) {
      gfo_state* st = &states[i];
      if (st->pending_calls < st->delay) continue;
      if (t > 0 && (c64 ? launch_move_finish<float2>(geos[i], st, lays[i], t - 1, stream)
                        : launch_move_finish<double2>(geos[i], st, lays[i], t - 1, stream)) !=
                       hipSuccess)
        return GFO_EHIP;
      if (launch_flush(geos[i], st, lays[i], stream) != hipSuccess) return GFO_EHIP;
      st->pending_calls = 0;
      flushed |= (uint64_t)1 << i;
    }
    if ((c64 ? launch_table_move<float2>(tab, n_jobs, wg_move, t, flushed, small, batch, stream)
             : launch_table_move<double2>(tab, n_jobs, wg_move, t, flushed, small, batch, stream)) !=
        hipSuccess)
      return GFO_EHIP;
    for (int i = 0; i < n_jobs; ++i) ++states[i].pending_calls;
  }
  if ((c64 ? launch_table_finish<float2>(tab, n_jobs, wg_finish, n_steps - 1, stream)
           : launch_table_finish<double2>(tab, n_jobs, wg_finish, n_steps - 1, stream)) != hipSuccess)
    return GFO_EHIP;
  for (int i = 0; i < n_jobs; ++i) {
    gfo_state* st = &states[i];
    if (st->pending_calls >= st->delay) {
      if (launch_flush(geos[i], st, lays[i], stream) != hipSuccess) return GFO_EHIP;
      st->pending_calls = 0;
    }
  }
  return GFO_OK;
}
