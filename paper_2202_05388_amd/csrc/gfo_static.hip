// score_candidates_static: score_candidates with its scratch in a file-scope
// device array instead of the caller's workspace, for callers that cannot
// allocate device memory.
//
// The array is a device symbol: its name in host code is a host-side stand-in,
// not a device address.  Its address on each device is taken once, with that
// device current, by hipGetSymbolAddress, and only that address is used from
// then on (kernel arguments).  Each device holds its own copy of the array
// until the process ends; every call on one device shares it, so calls that
// overlap on one device race.  Nothing in it needs clearing: the score kernel
// writes every entry that the selection kernel reads.
#include "gfo_internal.hpp"

#include <atomic>
#include <mutex>

namespace gfo {

static __device__ __align__(256) unsigned char scratch[GFO_STATIC_SCRATCH_BYTES];

// Layout inside the scratch: the workgroup summaries first, then the scores.
constexpr size_t kStaticPartial = 0;
constexpr size_t kStaticPfirst = kScoreMaxBlocks * sizeof(double);
constexpr size_t kStaticScores =
    (kStaticPfirst + kScoreMaxBlocks * sizeof(int) + 255) / 256 * 256;

constexpr int kMaxDevices = 64;
static std::atomic<unsigned char*> g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

// Device address of `scratch` on the current device (taken on first use).
static int scratch_address(unsigned char** out) {
  int dev = 0;
  if (note_hip(hipGetDevice(&dev)) != hipSuccess) return GFO_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return GFO_EINVAL;
  unsigned char* p = g_scratch_ptr[dev].load(std::memory_order_acquire);
  if (!p) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
    if (!p) {
      void* addr = nullptr;
      if (note_hip(hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch))) != hipSuccess || !addr)
        return GFO_EHIP;
      p = (unsigned char*)addr;
      g_scratch_ptr[dev].store(p, std::memory_order_release);
    }
  }
  *out = p;
  return GFO_OK;
}

size_t static_scratch_need(const gfo_problem* p) {
  return kStaticScores + (size_t)p->ny * p->nx * p->n_eps * sizeof(double);
}

}  // namespace gfo

using namespace gfo;

extern "C" int score_candidates_static(const gfo_problem* prob, const gfo_state* st,
                                       uint32_t cand_mask, double tau, int32_t topk,
                                       int32_t min_spacing, gfo_pick* d_out, hipStream_t stream) {
  discard_stale_hip();
  int rc = validate_problem(prob);
  if (rc) return rc;
  if ((rc = validate_state_fields(prob, st))) return rc;
  if (!d_out || topk < 1 || topk > GFO_MAX_RANK_K || min_spacing < 0 || !(tau >= 0.0) ||
      !(tau < 1.0))
    return GFO_EINVAL;
  const uint32_t mask = cand_mask & ((1u << prob->n_eps) - 1u);
  if (mask == 0) return GFO_EINVAL;
  if (static_scratch_need(prob) > GFO_STATIC_SCRATCH_BYTES) return GFO_ESCRATCH;
  unsigned char* base = nullptr;
  if ((rc = scratch_address(&base))) return rc;
  const ScoreBufs b{(double*)(base + kStaticScores), (double*)(base + kStaticPartial),
                    (int*)(base + kStaticPfirst)};
  const Geo g = make_geo(prob, st);
  if (launch_score_into(g, st, b, mask, tau, topk, min_spacing, d_out, stream) != hipSuccess)
    return GFO_EHIP;
  return GFO_OK;
}
