// p32_server.hip -- a request queue serving many Posit(32,2) linear systems
// of different sizes with continuous batching (the factor + solve service the
// batched routines make possible; the systems are those of the paper's LU and
// Cholesky study, Section 5, arriving one by one).
//
// Clients submit a system (A and B copied from host memory at submission) and
// later poll or wait for its solution.  One worker thread owns the device
// side:
//   * admission: requests are admitted in arrival order while their device
//     footprint (A, B, pivots) fits the pool the queue was created with; a
//     request that does not fit waits at the head of the queue until
//     completed requests free memory (no reordering, so no starvation);
//   * continuous batching: whenever fewer than two batches are in flight, the
//     worker takes every admitted request that is waiting (up to max_batch)
//     and launches it as one batch, without waiting for a batch to fill:
//     systems with n <= batch_max_n / 2 go through the batched kernels (one
//     launch per kind), and so do those with n <= batch_max_n when at least
//     kMidShare of them are in the batch; the others go through the
//     single-matrix routines, except that the new LU systems among them are
//     factored together (launch_getrf_group: their panels in one cooperative
//     launch per panel step, their trailing updates in one launch), and the
//     large Cholesky systems run by turns on kSideStreams side streams, so
//     large systems in one batch share the device instead of queueing behind
//     each other;
//   * overlap: a batch's host-to-device copies run on a copy stream while the
//     previous batch computes on the compute stream; results come back on the
//     compute stream and are copied out when its event completes;
//   * resident factors: a request may keep its factorisation on the device;
//     later requests then solve with it (no refactorisation) until it is
//     released.
// Every system is computed by the same routines as a standalone call, so a
// result is bit-identical whether it was served alone or in any batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "posit32.h"
#include "p32_launch.hpp"

namespace {

constexpr size_t kAlign = 256;
constexpr int kSlots = 2;                    // batches in flight
// A system with batch_max_n / 2 < n <= batch_max_n takes longer in one
// workgroup of the batched kernel than alone through the single-matrix
// routines (n = 512: about 20 ms against 5 ms), unless several of them share
// a batch and run side by side; they join the batched launch only when at
// least this many of them are in the batch.
constexpr size_t kMidShare = 4;
// Large Cholesky systems of a batch each go to one of these streams (by
// turns), so that their latency-bound column steps overlap on the device.
constexpr int kSideStreams = 4;

size_t round_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// first-fit sub-allocator over the device pool
struct Pool {
  size_t size = 0, used = 0;
  std::map<size_t, size_t> free_;            // offset -> length

  void init(size_t s) {
    size = s;
    used = 0;
    free_.clear();
    free_[0] = s;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = round_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t o = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[o + bytes] = rest;
      used += bytes;
      *off = o;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round_up(bytes);
    used -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
};

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

struct Factor {
  int32_t kind = 0;
  int64_t n = 0;
  size_t off = 0, bytes = 0;                 // A (factors) then ipiv
  int refs = 0;                              // requests in flight using it
  bool released = false;
};

struct Req {
  uint64_t ticket = 0;
  int32_t kind = 0;
  int64_t n = 0, nrhs = 0;
  uint64_t factor_in = 0;                    // solve with this resident factor
  bool keep = false;
  std::vector<uint32_t> A, B;                // host copies (A empty for factor_in)
  size_t fac_off = 0, fac_bytes = 0;         // device: A then ipiv (new systems)
  size_t rhs_off = 0, rhs_bytes = 0;         // device: B
  int32_t status = 1;                        // 1 pending / running, 0 done, < 0 error
  int32_t info = 0;
  uint64_t factor_out = 0;
  double t_submit = 0, t_start = 0, t_done = 0;
  size_t stage_x = 0;                        // offset of X in the slot's result staging
};

struct Slot {
  std::vector<Req*> reqs;
  char* pin_in = nullptr;                    // pinned: packed inputs and launch arrays
  size_t pin_in_cap = 0;
  char* pin_out = nullptr;                   // pinned: solutions and info
  size_t pin_out_cap = 0;
  char* dev_meta = nullptr;                  // device: launch arrays
  size_t dev_meta_cap = 0;
  hipEvent_t ev_in = nullptr, ev_done = nullptr;
  hipEvent_t ev_start = nullptr;             // compute stream: inputs and info ready
  hipEvent_t ev_side[kSideStreams] = {};     // side stream k: its systems done
  bool busy = false;
};

}  // namespace

struct posit32_queue {
  posit32_queue_cfg cfg{};
  p32::Tuning tune[2];                       // sub-panel tables: LU, Cholesky
  int device = 0;
  hipStream_t compute = nullptr, copy = nullptr;
  hipStream_t side[kSideStreams] = {};       // large Cholesky systems (default priority)
  char* dev_pool = nullptr;
  Pool pool;
  std::chrono::steady_clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> pending;
  std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
  std::unordered_map<uint64_t, Factor> factors;
  uint64_t next_ticket = 1, next_factor = 1;
  int64_t batches = 0, systems_done = 0;
  bool stop = false;
  Slot slots[kSlots];
  std::deque<int> inflight;                  // slot indices in launch order
  std::thread worker;
  int fatal = 0;                             // first HIP failure of the worker
};

namespace {

int hip_code(hipError_t e) { return e == hipSuccess ? 0 : P32_E_HIP - (int)e; }

int grow_pinned(char** p, size_t* cap, size_t need) {
  if (need <= *cap) return 0;
  if (*p) (void)hipHostFree(*p);
  *p = nullptr;
  *cap = 0;
  const size_t c = std::max(need, (size_t)1 << 20);
  const hipError_t e = hipHostMalloc((void**)p, c, hipHostMallocDefault);
  if (e != hipSuccess) return hip_code(e);
  *cap = c;
  return 0;
}

int grow_device(char** p, size_t* cap, size_t need) {
  if (need <= *cap) return 0;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  const size_t c = std::max(need, (size_t)1 << 16);
  const hipError_t e = hipMalloc((void**)p, c);
  if (e != hipSuccess) return hip_code(e);
  *cap = c;
  return 0;
}

__global__ void zero_info_kernel(int32_t* p, int32_t count) {
  for (int32_t i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0;
}

size_t factor_bytes(const Req& r) {
  return round_up((size_t)r.n * r.n * 4) + round_up((size_t)r.n * 4);
}

// A waiting request leaves the queue without running (lock held).
void drop_pending(posit32_queue* q, Req* r, int status) {
  if (r->factor_in) {
    Factor& f = q->factors.at(r->factor_in);
    f.refs -= 1;
    if (f.released && f.refs == 0) {
      q->pool.release(f.off, f.bytes);
      q->factors.erase(r->factor_in);
    }
  }
  r->A.clear();
  r->status = status;
}

// Admit waiting requests in order while they fit (called with the lock held).
std::vector<Req*> admit(posit32_queue* q) {
  std::vector<Req*> out;
  while (!q->pending.empty() && (int)out.size() < q->cfg.max_batch) {
    Req* r = q->pending.front();
    const size_t rb = round_up((size_t)r->n * r->nrhs * 4);
    size_t fo = 0, ro = 0;
    if (r->factor_in == 0) {
      if (!q->pool.alloc(factor_bytes(*r), &fo)) break;
      if (!q->pool.alloc(rb, &ro)) {
        q->pool.release(fo, factor_bytes(*r));
        break;
      }
      r->fac_off = fo;
      r->fac_bytes = factor_bytes(*r);
    } else {
      if (!q->pool.alloc(rb, &ro)) break;
      r->fac_off = q->factors.at(r->factor_in).off;
      r->fac_bytes = 0;                      // owned by the factor
    }
    r->rhs_off = ro;
    r->rhs_bytes = rb;
    q->pending.pop_front();
    out.push_back(r);
  }
  return out;
}

// Device work of one batch on the compute stream (inputs already copied).
int launch_batch(posit32_queue* q, Slot& s, const std::vector<Req*>& group, int kind, bool factor,
                 size_t meta_off, size_t info_off, int32_t max_n) {
  if (group.empty()) return 0;
  const int32_t count = (int32_t)group.size();
  char* m = s.dev_meta + meta_off;
  const int32_t* n = (const int32_t*)m;
  const int32_t* nrhs = (const int32_t*)(m + round_up(count * 4));
  const int64_t* lda = (const int64_t*)(m + 2 * round_up(count * 4));
  const int64_t* ldb = lda + count;
  uint32_t* const* A = (uint32_t* const*)(ldb + count);
  uint32_t* const* B = A + count;
  int32_t* const* ipiv = (int32_t* const*)(B + count);
  int32_t* info = (int32_t*)(s.dev_meta + info_off);
  if (factor)
    return p32::launch_vbatched(q->compute, kind, true, true, count, max_n, q->cfg.nb, n, A, lda,
                                kind == 0 ? ipiv : nullptr, nrhs, B, ldb, info, &q->tune[kind]);
  return p32::launch_vbatched(q->compute, kind, false, true, count, max_n, q->cfg.nb, n, A, lda,
                              kind == 0 ? ipiv : nullptr, nrhs, B, ldb, info, &q->tune[kind]);
}

// Stage, copy and launch one batch into slot s (without the lock).
int start_batch(posit32_queue* q, Slot& s) {
  std::vector<Req*>& rs = s.reqs;
  // largest systems first: the batched kernel's workgroups start in system order
  std::stable_sort(rs.begin(), rs.end(), [](const Req* a, const Req* b) { return a->n > b->n; });
  const int64_t small_max = q->cfg.batch_max_n, mid_min = small_max / 2;
  size_t mid = 0;
  for (const Req* r : rs) mid += r->n > mid_min && r->n <= small_max;
  const int64_t batched_max = mid >= kMidShare ? small_max : mid_min;
  // groups: 0 LU new, 1 Cholesky new, 2 LU resident, 3 Cholesky resident (batched)
  std::vector<Req*> groups[4], large;
  for (Req* r : rs) {
    if (r->n > batched_max) large.push_back(r);
    else groups[(r->factor_in ? 2 : 0) + r->kind].push_back(r);
  }
  // packed inputs
  size_t in_bytes = 0;
  for (Req* r : rs) in_bytes += round_up(r->A.size() * 4) + round_up(r->B.size() * 4);
  size_t meta_bytes = 0, meta_off[4];
  for (int g = 0; g < 4; ++g) {
    const size_t c = groups[g].size();
    meta_off[g] = meta_bytes;
    meta_bytes += 2 * round_up(c * 4) + round_up(c * 8 * 5);
  }
  const size_t info_off = meta_bytes;
  meta_bytes += round_up(rs.size() * 4);
  size_t out_bytes = round_up(rs.size() * 4);
  for (Req* r : rs) {
    r->stage_x = out_bytes;
    out_bytes += round_up((size_t)r->n * r->nrhs * 4);
  }
  int rc = grow_pinned(&s.pin_in, &s.pin_in_cap, in_bytes + meta_bytes);
  if (!rc) rc = grow_pinned(&s.pin_out, &s.pin_out_cap, out_bytes);
  if (!rc) rc = grow_device(&s.dev_meta, &s.dev_meta_cap, meta_bytes);
  if (rc) return rc;
  char* pool = q->dev_pool;
  size_t at = 0;
  for (Req* r : rs) {
    if (!r->A.empty()) {
      std::memcpy(s.pin_in + at, r->A.data(), r->A.size() * 4);
      rc = hip_code(hipMemcpyAsync(pool + r->fac_off, s.pin_in + at, r->A.size() * 4,
                                   hipMemcpyHostToDevice, q->copy));
      at += round_up(r->A.size() * 4);
    }
    std::memcpy(s.pin_in + at, r->B.data(), r->B.size() * 4);
    if (!rc)
      rc = hip_code(hipMemcpyAsync(pool + r->rhs_off, s.pin_in + at, r->B.size() * 4,
                                   hipMemcpyHostToDevice, q->copy));
    at += round_up(r->B.size() * 4);
    if (rc) return rc;
  }
  // launch arrays of each batched group
  char* meta = s.pin_in + in_bytes;
  for (int g = 0; g < 4; ++g) {
    const size_t c = groups[g].size();
    char* m = meta + meta_off[g];
    int32_t* n = (int32_t*)m;
    int32_t* nrhs = (int32_t*)(m + round_up(c * 4));
    int64_t* lda = (int64_t*)(m + 2 * round_up(c * 4));
    int64_t* ldb = lda + c;
    uint64_t* A = (uint64_t*)(ldb + c);
    uint64_t* B = A + c;
    uint64_t* ipiv = B + c;
    for (size_t i = 0; i < c; ++i) {
      const Req* r = groups[g][i];
      n[i] = (int32_t)r->n;
      nrhs[i] = (int32_t)r->nrhs;
      lda[i] = r->n;
      ldb[i] = r->nrhs;
      A[i] = (uint64_t)(pool + r->fac_off);
      B[i] = (uint64_t)(pool + r->rhs_off);
      ipiv[i] = (uint64_t)(pool + r->fac_off + round_up((size_t)r->n * r->n * 4));
    }
  }
  rc = hip_code(hipMemcpyAsync(s.dev_meta, meta, meta_bytes, hipMemcpyHostToDevice, q->copy));
  if (!rc) rc = hip_code(hipEventRecord(s.ev_in, q->copy));
  if (!rc) rc = hip_code(hipStreamWaitEvent(q->compute, s.ev_in, 0));
  if (rc) return rc;
  const double t = now_s(q->t0);
  for (Req* r : rs) r->t_start = t;
  // info array of the batch: the batched groups in order, then the large
  // systems; r->info holds the request's index into it until the batch ends
  int32_t* dinfo = (int32_t*)(s.dev_meta + info_off);
  int32_t sub = 0;
  for (int g = 0; g < 4 && !rc; ++g) {
    int32_t max_n = 0;
    for (Req* r : groups[g]) {
      max_n = std::max(max_n, (int32_t)r->n);
      r->info = sub++;
    }
    rc = launch_batch(q, s, groups[g], g & 1, g < 2, meta_off[g],
                      info_off + (size_t)(sub - (int32_t)groups[g].size()) * 4, max_n);
  }
  if (!rc && !large.empty()) {
    // single-matrix routines; their info goes to the same array (a resident
    // factor was checked when it was kept, so its solve reports 0)
    hipLaunchKernelGGL(zero_info_kernel, dim3(1), dim3(256), 0, q->compute, dinfo + sub,
                       (int32_t)large.size());
    rc = p32::launch_status();
  }
  // the large Cholesky systems, by turns on the side streams, which first
  // wait for everything queued on the compute stream so far (inputs, info
  // zeroing); the compute stream waits for them before the results are
  // copied out
  int sides = 0;
  {
    size_t nchol = 0;
    for (Req* r : large) nchol += r->kind == 1;
    sides = (int)std::min(nchol, (size_t)kSideStreams);
  }
  if (!rc && sides > 0) {
    rc = hip_code(hipEventRecord(s.ev_start, q->compute));
    for (int k = 0; k < sides && !rc; ++k) rc = hip_code(hipStreamWaitEvent(q->side[k], s.ev_start, 0));
    int turn = 0;
    for (size_t i = 0; i < large.size() && !rc; ++i) {
      Req* r = large[i];
      if (r->kind != 1) continue;
      hipStream_t st = q->side[turn++ % sides];
      uint32_t* A = (uint32_t*)(pool + r->fac_off);
      uint32_t* B = (uint32_t*)(pool + r->rhs_off);
      int32_t* info = dinfo + sub + (int32_t)i;
      if (!r->factor_in) rc = p32::launch_potrf(st, 0, r->n, q->cfg.nb, A, r->n, info);
      if (!rc) rc = p32::launch_potrs(st, 0, r->n, r->nrhs, A, r->n, B, r->nrhs);
    }
    for (int k = 0; k < sides && !rc; ++k) rc = hip_code(hipEventRecord(s.ev_side[k], q->side[k]));
  }
  // the new LU systems among them are factored together, up to
  // kGetrfGroupMax at a time (their panels share the per-column latency)
  std::vector<Req*> lu_new;
  for (Req* r : large)
    if (r->kind == 0 && !r->factor_in) lu_new.push_back(r);
  for (size_t g0 = 0; g0 < lu_new.size() && !rc; g0 += p32::kGetrfGroupMax) {
    const int c = (int)std::min(lu_new.size() - g0, (size_t)p32::kGetrfGroupMax);
    int64_t n[p32::kGetrfGroupMax], lda[p32::kGetrfGroupMax];
    uint32_t* A[p32::kGetrfGroupMax];
    int32_t* ipiv[p32::kGetrfGroupMax];
    int32_t* info[p32::kGetrfGroupMax];
    for (int i = 0; i < c; ++i) {
      Req* r = lu_new[g0 + i];
      n[i] = lda[i] = r->n;
      A[i] = (uint32_t*)(pool + r->fac_off);
      ipiv[i] = (int32_t*)(pool + r->fac_off + round_up((size_t)r->n * r->n * 4));
      info[i] = dinfo + sub + (int32_t)(std::find(large.begin(), large.end(), r) - large.begin());
    }
    rc = p32::launch_getrf_group(q->compute, c, n, q->cfg.nb, A, lda, ipiv, info);
  }
  // and all their solves (new and resident factors) go together too
  std::vector<Req*> lu_all;
  for (Req* r : large)
    if (r->kind == 0) lu_all.push_back(r);
  for (size_t g0 = 0; g0 < lu_all.size() && !rc; g0 += p32::kGetrfGroupMax) {
    const int c = (int)std::min(lu_all.size() - g0, (size_t)p32::kGetrfGroupMax);
    int64_t n[p32::kGetrfGroupMax], nrhs[p32::kGetrfGroupMax], ld[p32::kGetrfGroupMax];
    const uint32_t* LU[p32::kGetrfGroupMax];
    const int32_t* ipiv[p32::kGetrfGroupMax];
    uint32_t* B[p32::kGetrfGroupMax];
    for (int i = 0; i < c; ++i) {
      Req* r = lu_all[g0 + i];
      n[i] = r->n;
      nrhs[i] = r->nrhs;
      ld[i] = r->n;
      LU[i] = (const uint32_t*)(pool + r->fac_off);
      ipiv[i] = (const int32_t*)(pool + r->fac_off + round_up((size_t)r->n * r->n * 4));
      B[i] = (uint32_t*)(pool + r->rhs_off);
    }
    // right-hand sides in the ldb array (B is n x nrhs, row stride nrhs)
    rc = p32::launch_getrs_group(q->compute, c, n, nrhs, LU, ld, ipiv, B, nrhs);
  }
  for (Req* r : large) r->info = sub++;           // LU above, Cholesky on the side streams
  for (int k = 0; k < sides && !rc; ++k) rc = hip_code(hipStreamWaitEvent(q->compute, s.ev_side[k], 0));
  if (rc) return rc;
  // results: info array, then each solution
  rc = hip_code(hipMemcpyAsync(s.pin_out, s.dev_meta + info_off, rs.size() * 4, hipMemcpyDeviceToHost,
                               q->compute));
  for (Req* r : rs) {
    if (rc) break;
    rc = hip_code(hipMemcpyAsync(s.pin_out + r->stage_x, pool + r->rhs_off,
                                 (size_t)r->n * r->nrhs * 4, hipMemcpyDeviceToHost, q->compute));
  }
  if (!rc) rc = hip_code(hipEventRecord(s.ev_done, q->compute));
  return rc;
}

// Results of a completed batch (lock held).
void finish_batch(posit32_queue* q, Slot& s, int rc) {
  const double t = now_s(q->t0);
  const int32_t* infos = (const int32_t*)s.pin_out;
  for (Req* r : s.reqs) {
    const int32_t info = rc ? 0 : infos[r->info];
    r->info = info;
    if (rc) {
      r->status = rc;
    } else {
      // a failed factorisation is not solved: X is the submitted B (the
      // single-matrix routines of large systems ran their solve regardless)
      if (info == 0)
        r->B.assign((const uint32_t*)(s.pin_out + r->stage_x),
                    (const uint32_t*)(s.pin_out + r->stage_x) + (size_t)r->n * r->nrhs);
      r->status = 0;
    }
    r->A.clear();
    r->A.shrink_to_fit();
    q->pool.release(r->rhs_off, r->rhs_bytes);
    if (r->factor_in) {
      Factor& f = q->factors.at(r->factor_in);
      f.refs -= 1;
      if (f.released && f.refs == 0) {
        q->pool.release(f.off, f.bytes);
        q->factors.erase(r->factor_in);
      }
    } else if (r->keep && rc == 0 && info == 0) {
      Factor f;
      f.kind = r->kind;
      f.n = r->n;
      f.off = r->fac_off;
      f.bytes = r->fac_bytes;
      r->factor_out = q->next_factor++;
      q->factors[r->factor_out] = f;
    } else {
      q->pool.release(r->fac_off, r->fac_bytes);
    }
    r->t_done = t;
    q->systems_done += 1;
  }
  s.reqs.clear();
  s.busy = false;
  q->cv_done.notify_all();
}

void worker_main(posit32_queue* q) {
  (void)hipSetDevice(q->device);
  std::unique_lock<std::mutex> lk(q->mu);
  for (;;) {
    // completed batches, oldest first
    while (!q->inflight.empty()) {
      Slot& s = q->slots[q->inflight.front()];
      const hipError_t e = hipEventQuery(s.ev_done);
      if (e == hipErrorNotReady) break;
      q->inflight.pop_front();
      const int rc = hip_code(e);
      if (rc && !q->fatal) q->fatal = rc;
      finish_batch(q, s, rc);
    }
    if (q->stop && q->pending.empty() && q->inflight.empty()) break;
    // a new batch when a slot is free and something is admissible
    int free_slot = -1;
    for (int i = 0; i < kSlots; ++i)
      if (!q->slots[i].busy) free_slot = i;
    if (free_slot >= 0 && !q->pending.empty() && !q->fatal) {
      std::vector<Req*> batch = admit(q);
      if (!batch.empty()) {
        Slot& s = q->slots[free_slot];
        s.busy = true;
        s.reqs = std::move(batch);
        q->batches += 1;
        lk.unlock();
        const int rc = start_batch(q, s);
        lk.lock();
        if (rc) {
          if (!q->fatal) q->fatal = rc;
          (void)hipStreamSynchronize(q->compute);
          for (hipStream_t st : q->side) (void)hipStreamSynchronize(st);
          finish_batch(q, s, rc);
        } else {
          q->inflight.push_back(free_slot);
        }
        continue;
      }
      if (q->inflight.empty()) {
        // the head of the queue does not fit an empty pool: it never will
        Req* r = q->pending.front();
        q->pending.pop_front();
        drop_pending(q, r, P32_E_NOMEM);
        q->cv_done.notify_all();
        continue;
      }
    }
    if (q->fatal) {
      // fail whatever is still waiting once the device has failed
      while (!q->pending.empty()) {
        drop_pending(q, q->pending.front(), q->fatal);
        q->pending.pop_front();
      }
      q->cv_done.notify_all();
    }
    if (!q->inflight.empty()) {
      // poll the oldest batch, waking early for new arrivals
      q->cv_work.wait_for(lk, std::chrono::microseconds(50));
    } else {
      q->cv_work.wait(lk, [q] { return q->stop || !q->pending.empty(); });
    }
  }
}

}  // namespace

extern "C" {

int posit32_queue_create(const posit32_queue_cfg* cfg, posit32_queue** out) {
  if (cfg == nullptr || out == nullptr) return -1;
  if (cfg->device_bytes < (1 << 20)) return -1;
  if (cfg->max_batch < 1) return -1;
  if (cfg->nb < 1 || cfg->nb > 256) return -1;
  if (cfg->batch_max_n < 0) return -1;
  if (cfg->max_pending < 0) return -1;
  auto q = std::make_unique<posit32_queue>();
  for (int kind = 0; kind < 2; ++kind) {
    if (cfg->tuning == nullptr) q->tune[kind] = p32::default_tuning(kind);
    else if (p32::tuning_from_abi(cfg->tuning[kind], &q->tune[kind])) return -1;
  }
  q->cfg = *cfg;
  q->cfg.tuning = nullptr;                   // the tables were copied
  q->t0 = std::chrono::steady_clock::now();
  int rc = hip_code(hipGetDevice(&q->device));
  if (!rc) rc = hip_code(hipStreamCreateWithFlags(&q->compute, hipStreamNonBlocking));
  if (!rc) rc = hip_code(hipStreamCreateWithFlags(&q->copy, hipStreamNonBlocking));
  for (int k = 0; k < kSideStreams && !rc; ++k)
    rc = hip_code(hipStreamCreateWithFlags(&q->side[k], hipStreamNonBlocking));
  if (!rc) rc = hip_code(hipMalloc((void**)&q->dev_pool, (size_t)cfg->device_bytes));
  for (int i = 0; i < kSlots && !rc; ++i) {
    rc = hip_code(hipEventCreateWithFlags(&q->slots[i].ev_in, hipEventDisableTiming));
    if (!rc) rc = hip_code(hipEventCreateWithFlags(&q->slots[i].ev_done, hipEventDisableTiming));
    if (!rc) rc = hip_code(hipEventCreateWithFlags(&q->slots[i].ev_start, hipEventDisableTiming));
    for (int k = 0; k < kSideStreams && !rc; ++k)
      rc = hip_code(hipEventCreateWithFlags(&q->slots[i].ev_side[k], hipEventDisableTiming));
  }
  if (rc) {
    posit32_queue_destroy(q.release());
    return rc;
  }
  q->pool.init((size_t)cfg->device_bytes);
  posit32_queue* raw = q.release();
  raw->worker = std::thread(worker_main, raw);
  *out = raw;
  return 0;
}

int posit32_queue_submit(posit32_queue* q, const posit32_request* req, uint64_t* ticket) {
  if (q == nullptr) return -1;
  if (req == nullptr || ticket == nullptr) return -2;
  if (req->kind != P32_REQ_LU && req->kind != P32_REQ_CHOL) return -2;
  if (req->n < 1 || req->n > 0xFFFFFE || req->nrhs < 1) return -2;
  if (req->B == nullptr || (req->factor == 0 && req->A == nullptr)) return -2;
  auto r = std::make_unique<Req>();
  r->kind = req->kind;
  r->n = req->n;
  r->nrhs = req->nrhs;
  r->factor_in = req->factor;
  r->keep = req->keep != 0 && req->factor == 0;
  const size_t nn = (size_t)req->n * req->n, nb = (size_t)req->n * req->nrhs;
  std::lock_guard<std::mutex> lk(q->mu);
  if (q->stop) return -1;
  if (q->cfg.max_pending > 0 && (int64_t)q->reqs.size() >= q->cfg.max_pending) return P32_E_BUSY;
  if (req->factor) {
    auto it = q->factors.find(req->factor);
    if (it == q->factors.end() || it->second.released || it->second.kind != req->kind ||
        it->second.n != req->n)
      return -2;
    it->second.refs += 1;                    // held until this request completes
  } else {
    const size_t need = factor_bytes(*r) + round_up(nb * 4);
    if (need > q->pool.size) return P32_E_NOMEM;   // larger than the whole pool
    r->A.assign(req->A, req->A + nn);
  }
  r->B.assign(req->B, req->B + nb);
  r->ticket = q->next_ticket++;
  r->t_submit = now_s(q->t0);
  *ticket = r->ticket;
  q->pending.push_back(r.get());
  q->reqs[r->ticket] = std::move(r);
  q->cv_work.notify_one();
  return 0;
}

static int take_result(posit32_queue* q, Req* r, posit32_t* X, posit32_result* res) {
  res->status = r->status;
  res->info = r->info;
  res->factor = r->factor_out;
  res->submit_s = r->t_submit;
  res->start_s = r->t_start;
  res->done_s = r->t_done;
  if (r->status == 1) return 1;
  if (r->status == 0 && X != nullptr) std::memcpy(X, r->B.data(), r->B.size() * 4);
  const int st = r->status;
  q->reqs.erase(r->ticket);
  return st;
}

int posit32_queue_poll(posit32_queue* q, uint64_t ticket, posit32_t* X, posit32_result* res) {
  if (q == nullptr) return -1;
  if (res == nullptr) return -4;
  std::lock_guard<std::mutex> lk(q->mu);
  auto it = q->reqs.find(ticket);
  if (it == q->reqs.end()) return -2;
  return take_result(q, it->second.get(), X, res);
}

int posit32_queue_wait(posit32_queue* q, uint64_t ticket, double timeout_s, posit32_t* X,
                       posit32_result* res) {
  if (q == nullptr) return -1;
  if (res == nullptr) return -5;
  std::unique_lock<std::mutex> lk(q->mu);
  auto it = q->reqs.find(ticket);
  if (it == q->reqs.end()) return -2;
  Req* r = it->second.get();
  const auto until = std::chrono::steady_clock::now() +
                     std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                         std::chrono::duration<double>(timeout_s < 0 ? 1e9 : timeout_s));
  q->cv_done.wait_until(lk, until, [r] { return r->status != 1; });
  return take_result(q, r, X, res);
}

int posit32_factor_release(posit32_queue* q, uint64_t factor) {
  if (q == nullptr) return -1;
  std::lock_guard<std::mutex> lk(q->mu);
  auto it = q->factors.find(factor);
  if (it == q->factors.end() || it->second.released) return -2;
  it->second.released = true;
  if (it->second.refs == 0) {
    q->pool.release(it->second.off, it->second.bytes);
    q->factors.erase(it);
  }
  return 0;
}

int posit32_queue_stats(posit32_queue* q, posit32_queue_stats_t* st) {
  if (q == nullptr) return -1;
  if (st == nullptr) return -2;
  std::lock_guard<std::mutex> lk(q->mu);
  st->pending = (int64_t)q->pending.size();
  st->inflight_batches = (int64_t)q->inflight.size();
  st->batches = q->batches;
  st->systems_done = q->systems_done;
  st->pool_bytes = (int64_t)q->pool.size;
  st->pool_used = (int64_t)q->pool.used;
  st->resident_factors = (int64_t)q->factors.size();
  st->error = q->fatal;
  return 0;
}

int posit32_queue_destroy(posit32_queue* q) {
  if (q == nullptr) return -1;
  {
    std::lock_guard<std::mutex> lk(q->mu);
    q->stop = true;
  }
  q->cv_work.notify_all();
  if (q->worker.joinable()) q->worker.join();
  (void)hipSetDevice(q->device);
  for (Slot& s : q->slots) {
    if (s.pin_in) (void)hipHostFree(s.pin_in);
    if (s.pin_out) (void)hipHostFree(s.pin_out);
    if (s.dev_meta) (void)hipFree(s.dev_meta);
    if (s.ev_in) (void)hipEventDestroy(s.ev_in);
    if (s.ev_done) (void)hipEventDestroy(s.ev_done);
    if (s.ev_start) (void)hipEventDestroy(s.ev_start);
    for (hipEvent_t e : s.ev_side)
      if (e) (void)hipEventDestroy(e);
  }
  for (hipStream_t st : q->side)
    if (st) (void)hipStreamSynchronize(st);
  if (q->dev_pool) (void)hipFree(q->dev_pool);
  if (q->compute) (void)hipStreamDestroy(q->compute);
  if (q->copy) (void)hipStreamDestroy(q->copy);
  for (hipStream_t st : q->side)
    if (st) (void)hipStreamDestroy(st);
  delete q;
  return 0;
}

}  // extern "C"
