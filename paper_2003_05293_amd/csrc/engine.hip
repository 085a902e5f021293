// Serving engine of libhg (include/hg.h, hg_engine_*): continuous batching of
// hologram requests.  Every step advances each admitted hologram by one
// iteration of the paper's schedule (section 2) in one batched launch;
// requests join and leave between steps.  The per-hologram launch geometry
// is that of a batch of one, so results do not depend on the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "hg.h"
#include "kernels.hpp"
#include "runtime.hpp"

namespace {

using hg::set_error;

// First-fit allocator over [0, size) with 256-byte granules.
class PoolAllocator {
 public:
  void reset(size_t size) {
    free_.clear();
    free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) / 256 * 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t next = it->first + bytes;
      free_.erase(it);
      if (rest) free_[next] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
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

 private:
  std::map<size_t, size_t> free_;  // offset -> length
};

struct Request {
  uint64_t ticket = 0;
  hg::JobSpec spec;
  std::vector<double> spots;  // host copy of x, y, z, amp (host-resident inputs)
};

enum TicketState { kQueued = 0, kActive = 1, kFinishing = 2, kDone = 3 };

struct Slot {
  bool used = false;
  Request req;
  hg::JobLayout layout;
  hg::JobDev dev;
  size_t off = 0;
  int next_it = 1;            // next iteration to run (1-based)
  bool finishing = false;     // final phase enqueued; waiting for `done`
  hipEvent_t done = nullptr;  // recorded after the final phase
};

hg_status spec_from_job(const hg_job& j, hg::JobSpec* out) {
  if (!(j.compression > 0.0 && j.compression <= 1.0))
    return set_error(HG_EINVAL, "compression must be in (0, 1]");
  if (j.flags & ~(HG_PREC_MASK | HG_SPOTS_ON_DEVICE | HG_FULL_DIRECT))
    return set_error(HG_EINVAL, "flags: unknown bits set");
  const uint32_t prec = j.flags & HG_PREC_MASK;
  if (prec != HG_PREC_FP32 && prec != HG_PREC_MIXED)
    return set_error(HG_EINVAL, "flags: precision must be HG_PREC_FP32 or HG_PREC_MIXED");
  if (prec == HG_PREC_MIXED && (j.flags & HG_FULL_DIRECT))
    return set_error(HG_EINVAL, "flags: HG_FULL_DIRECT applies to HG_PREC_FP32 only");
  if (j.trace_V) return set_error(HG_EINVAL, "engine requests cannot ask for a trace");
  if (!j.phi_dev) return set_error(HG_EINVAL, "phi_dev must be non-NULL");
  HG_TRY(hg::make_spec(&j.grid, &j.optics, &j.spots, j.iterations, j.compression, j.seed,
                       j.flags, j.phi_dev, nullptr, out));
  HG_TRY(hg::apply_lut(j.lut, j.gray_dev, out));
  return hg::attach_shared_order(out);
}

}  // namespace

struct hg_engine {
  int device = 0;
  size_t budget = 0;
  int max_slots = 0;
  hg::TuneParams tp;
  std::mutex mu;
  hg::DevBuf<char> pool;
  PoolAllocator alloc;
  hg::DevBuf<int32_t> status;
  hg::DevBuf<char> step_buf;  // slot table, new-job table, descriptors
  hg::Staging staging;
  std::vector<Slot> slots;
  std::deque<Request> queue;
  std::map<uint64_t, int> state;  // ticket -> TicketState
  std::map<uint64_t, int> where;  // ticket -> slot (active / finishing)
  uint64_t next_ticket = 1;
  std::vector<hipEvent_t> event_pool;
  hipEvent_t step_events[2] = {nullptr, nullptr};
  bool step_pending[2] = {false, false};
  int step_index = 0;

  hipEvent_t get_event() {
    if (!event_pool.empty()) {
      hipEvent_t e = event_pool.back();
      event_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
  }

  // Frees the slot of a finished request once the device is done with it.
  bool try_retire(int si) {
    Slot& s = slots[si];
    if (!s.finishing) return false;
    if (hipEventQuery(s.done) != hipSuccess) return false;
    event_pool.push_back(s.done);
    alloc.release(s.off, s.layout.bytes);
    state[s.req.ticket] = kDone;
    where.erase(s.req.ticket);
    s = Slot{};
    return true;
  }
};

extern "C" {

hg_status hg_engine_create(const hg_engine_config* cfg, hg_engine** out) {
  if (!cfg || !out) return set_error(HG_EINVAL, "config and out must be non-NULL");
  if (cfg->max_slots < 1 || cfg->max_slots > HG_MAX_SPOTS)
    return set_error(HG_EINVAL, "max_slots must be in [1, 4096]");
  if (cfg->mem_budget_bytes < (size_t)(1 << 20))
    return set_error(HG_EINVAL, "mem_budget_bytes must be at least 1 MiB");
  if (cfg->tune.full_block_cap < 0 || cfg->tune.subset_block_cap < 0 ||
      cfg->tune.pass_form < 0 || cfg->tune.pass_form > 1 ||
      cfg->tune.chain_passes < 0 || cfg->tune.chain_passes > 1)
    return set_error(HG_EINVAL, "tune caps must be >= 0, pass_form and chain_passes 0 or 1");
  auto e = std::make_unique<hg_engine>();
  HG_HIP(hipGetDevice(&e->device));
  e->budget = cfg->mem_budget_bytes;
  e->max_slots = cfg->max_slots;
  if (cfg->tune.full_block_cap > 0) e->tp.full_block_cap = cfg->tune.full_block_cap;
  if (cfg->tune.subset_block_cap > 0) e->tp.subset_block_cap = cfg->tune.subset_block_cap;
  e->tp.pass_form = cfg->tune.pass_form;
  HG_TRY(e->pool.reserve(e->budget));
  e->alloc.reset(e->budget);
  HG_TRY(e->status.reserve(1));
  HG_HIP(hipMemset(e->status.p, 0, sizeof(int32_t)));
  e->slots.resize(e->max_slots);
  for (auto& ev : e->step_events) HG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  *out = e.release();
  return HG_OK;
}

hg_status hg_engine_submit(hg_engine* e, const hg_job* job, uint64_t* ticket) {
  if (!e || !job || !ticket) return set_error(HG_EINVAL, "engine, job and ticket must be non-NULL");
  Request r;
  HG_TRY(spec_from_job(*job, &r.spec));
  std::lock_guard<std::mutex> lk(e->mu);
  if (hg::layout_job(r.spec, e->tp, nullptr, true).bytes > e->budget)
    return set_error(HG_ENOMEM, "request needs more scratch than the engine's whole budget");
  if (!r.spec.spots_on_device) {
    const int N = r.spec.N;
    r.spots.resize(4 * (size_t)N);
    std::memcpy(r.spots.data(), r.spec.x, sizeof(double) * N);
    std::memcpy(r.spots.data() + N, r.spec.y, sizeof(double) * N);
    std::memcpy(r.spots.data() + 2 * N, r.spec.z, sizeof(double) * N);
    std::memcpy(r.spots.data() + 3 * N, r.spec.amp, sizeof(double) * N);
    r.spec.x = r.spec.y = r.spec.z = r.spec.amp = nullptr;
  }
  r.ticket = e->next_ticket++;
  *ticket = r.ticket;
  e->state[r.ticket] = kQueued;
  e->queue.push_back(std::move(r));
  return HG_OK;
}

hg_status hg_engine_step(hg_engine* e, void* stream, int32_t* pending_out) {
  if (!e) return set_error(HG_EINVAL, "engine must be non-NULL");
  std::lock_guard<std::mutex> lk(e->mu);
  hipStream_t s = (hipStream_t)stream;
  // at most two steps in flight
  const int k = e->step_index & 1;
  if (e->step_pending[k]) {
    HG_HIP(hipEventSynchronize(e->step_events[k]));
    e->step_pending[k] = false;
  }
  for (int si = 0; si < e->max_slots; ++si) e->try_retire(si);

  // admission, in arrival order, while a slot and pool room are free
  std::vector<int> fresh;
  while (!e->queue.empty()) {
    int free_slot = -1;
    for (int si = 0; si < e->max_slots; ++si)
      if (!e->slots[si].used) {
        free_slot = si;
        break;
      }
    if (free_slot < 0) break;
    Request& r = e->queue.front();
    hg::JobLayout L = hg::layout_job(r.spec, e->tp, e->status.p, true);
    size_t off = 0;
    if (!e->alloc.alloc(L.bytes, &off)) break;
    Slot& sl = e->slots[free_slot];
    sl.used = true;
    sl.req = std::move(r);
    e->queue.pop_front();
    sl.layout = L;
    sl.off = off;
    sl.dev = hg::bind_job(L, sl.req.spec, e->pool.p + off, nullptr);
    sl.next_it = 1;
    sl.finishing = false;
    e->state[sl.req.ticket] = kActive;
    e->where[sl.req.ticket] = free_slot;
    fresh.push_back(free_slot);
  }

  // step payload: [slot table][new jobs][perm slices][prologue slices]
  // [iteration][final][spots]
  std::vector<hg::JobDev> table(e->max_slots, hg::JobDev{});
  for (int si = 0; si < e->max_slots; ++si)
    if (e->slots[si].used) table[si] = e->slots[si].dev;
  std::vector<hg::JobDev> newjobs;
  std::vector<hg::JobSlice> perm;
  std::vector<hg::PrologueSlice> pro;
  int perm_blocks = 0, pro_blocks = 0;
  bool perm_lds = true;
  for (int si : fresh) {
    const hg::JobDev& j = e->slots[si].dev;
    if (j.compressed && !j.order_shared) {
      perm.push_back(hg::JobSlice{perm_blocks, (int32_t)newjobs.size()});
      perm_blocks += hg::perm_blocks(j.P);
      if (j.h > 11) perm_lds = false;
    }
    const hg::PrologueSlice ps{pro_blocks, (int32_t)newjobs.size(), hg::prologue_setup_blocks(j),
                               hg::prologue_table_blocks(j)};
    pro.push_back(ps);
    pro_blocks += ps.setup_blocks + ps.table_blocks;
    newjobs.push_back(j);
  }
  hg::LaunchSet iter, fin;
  std::vector<int> finishing;
  for (int si = 0; si < e->max_slots; ++si) {
    Slot& sl = e->slots[si];
    if (!sl.used || sl.finishing) continue;
    const hg::JobDev& j = sl.dev;
    if (sl.next_it <= j.iterations) {
      iter.add_iteration(j, sl.layout, sl.next_it, si);
      sl.next_it += 1;
    }
    if (sl.next_it > j.iterations) {
      fin.add_final(j, sl.layout, si);
      finishing.push_back(si);
    }
  }

  auto align = [](size_t v) { return (v + 255) / 256 * 256; };
  size_t o = 0;
  const size_t o_table = o;
  o = align(o + sizeof(hg::JobDev) * table.size());
  const size_t o_new = o;
  o = align(o + sizeof(hg::JobDev) * newjobs.size());
  const size_t o_perm = o;
  o = align(o + sizeof(hg::JobSlice) * perm.size());
  const size_t o_pro = o;
  o = align(o + sizeof(hg::PrologueSlice) * pro.size());
  const size_t o_iter = o;
  o += iter.bytes();
  const size_t o_fin = o;
  o += fin.bytes();
  const size_t table_bytes = o;
  size_t spot_bytes = 0;
  for (int si : fresh)
    if (!e->slots[si].req.spec.spots_on_device)
      spot_bytes += sizeof(double) * e->slots[si].req.spots.size();
  HG_TRY(e->step_buf.reserve(table_bytes));
  HG_TRY(e->staging.acquire(table_bytes + spot_bytes));
  char* st = e->staging.p;
  std::memcpy(st + o_table, table.data(), sizeof(hg::JobDev) * table.size());
  if (!newjobs.empty()) std::memcpy(st + o_new, newjobs.data(), sizeof(hg::JobDev) * newjobs.size());
  if (!perm.empty()) std::memcpy(st + o_perm, perm.data(), sizeof(hg::JobSlice) * perm.size());
  if (!pro.empty()) std::memcpy(st + o_pro, pro.data(), sizeof(hg::PrologueSlice) * pro.size());
  iter.stage(st + o_iter, e->step_buf.p + o_iter);
  fin.stage(st + o_fin, e->step_buf.p + o_fin);
  HG_HIP(hipMemcpyAsync(e->step_buf.p, st, table_bytes, hipMemcpyHostToDevice, s));
  size_t so = table_bytes;
  for (int si : fresh) {
    Slot& sl = e->slots[si];
    if (sl.req.spec.spots_on_device) continue;
    const size_t nb = sizeof(double) * sl.req.spots.size();
    std::memcpy(st + so, sl.req.spots.data(), nb);
    HG_HIP(hipMemcpyAsync(e->pool.p + sl.off + sl.layout.off_raw, st + so, nb,
                          hipMemcpyHostToDevice, s));
    so += nb;
  }
  HG_TRY(e->staging.mark_copied(s));
  const hg::JobDev* slots_dev = reinterpret_cast<const hg::JobDev*>(e->step_buf.p + o_table);
  if (!newjobs.empty()) {
    const hg::JobDev* new_dev = reinterpret_cast<const hg::JobDev*>(e->step_buf.p + o_new);
    hg::timed(s, "k_prologue", [&] {
      hg::launch_prologue(new_dev, reinterpret_cast<const hg::PrologueSlice*>(e->step_buf.p + o_pro),
                          (int)pro.size(), pro_blocks, s);
    });
    if (perm_blocks)
      hg::timed(s, "k_perm", [&] {
        hg::launch_perm_batch(new_dev, reinterpret_cast<const hg::JobSlice*>(e->step_buf.p + o_perm),
                              (int)perm.size(), perm_blocks, perm_lds, s);
      });
  }
  iter.launch(slots_dev, s, false);
  fin.launch(slots_dev, s, false);
  const hipError_t le = hipGetLastError();
  if (le != hipSuccess)
    return set_error(HG_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(le));
  for (int si : finishing) {
    Slot& sl = e->slots[si];
    sl.done = e->get_event();
    if (!sl.done) return set_error(HG_EDEVICE, "event creation failed");
    HG_HIP(hipEventRecord(sl.done, s));
    sl.finishing = true;
    e->state[sl.req.ticket] = kFinishing;
  }
  HG_HIP(hipEventRecord(e->step_events[k], s));
  e->step_pending[k] = true;
  e->step_index += 1;
  if (pending_out) {
    int32_t n = (int32_t)e->queue.size();
    for (const Slot& sl : e->slots) n += sl.used ? 1 : 0;
    *pending_out = n;
  }
  return HG_OK;
}

hg_status hg_engine_poll(hg_engine* e, uint64_t ticket, int32_t* done) {
  if (!e || !done) return set_error(HG_EINVAL, "engine and done must be non-NULL");
  std::lock_guard<std::mutex> lk(e->mu);
  auto it = e->state.find(ticket);
  if (it == e->state.end()) return set_error(HG_EINVAL, "unknown ticket");
  if (it->second == kFinishing) e->try_retire(e->where[ticket]);
  *done = e->state[ticket] == kDone ? 1 : 0;
  return HG_OK;
}

hg_status hg_engine_destroy(hg_engine* e) {
  if (!e) return HG_OK;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    int cur = 0;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    (void)hipSetDevice(e->device);
    (void)hipDeviceSynchronize();
    for (Slot& sl : e->slots)
      if (sl.done) (void)hipEventDestroy(sl.done);
    for (hipEvent_t ev : e->event_pool) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : e->step_events)
      if (ev) (void)hipEventDestroy(ev);
    e->staging.release();
    e->step_buf.release();
    e->pool.release();
    e->status.release();
    if (have_cur) (void)hipSetDevice(cur);
  }
  delete e;
  return HG_OK;
}

}  // extern "C"
