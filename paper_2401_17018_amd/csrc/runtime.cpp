// Host runtime behind the C ABI (include/gamma.h): context, device memory,
// graph loading, query registration and the per-batch pipeline.
//
// Per batch (the four components of Sec. IV-A, with the search kernel of
// Sec. IV-C): canonicalise the batch and build the batch hash, delta-merge
// the touched rows, refresh the candidate filter of the touched vertices,
// generate seeds, search, commit G', refresh the filter again, return the
// results.  Every step is a HIP kernel on the context stream; the host only
// sizes buffers (one synchronisation after canonicalisation, before
// anything is mutated) and copies the small results back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/gamma.h"
#include "ctx_access.h"
#include "dev_common.h"
#include "host_plan.h"
#include "kernels.h"

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct DeviceError {
  hipError_t e;
  const char* what;
};
struct StatusError {
  gamma_status s;
  std::string msg;
};

inline void chk(hipError_t e, const char* what) {
  if (e != hipSuccess) throw DeviceError{e, what};
}

int bits_for(uint64_t x) {  // bits to hold any value < x (at least 1)
  int b = 1;
  while (b < 63 && (1ull << b) < x) ++b;
  return b;
}

// Device memory of gamma_apply_batch_noalloc: every per-batch buffer of that
// entry point (staged inputs, canonical batch, batch hash, sort and scan
// space, merge bookkeeping, seeds, counters, hand-over mailboxes, per-query
// and per-update results) is carved from this array.  Each GPU the library
// runs on holds its own copy until the process ends.  Host code never passes
// the array's name to the device: scratch_attach() looks up its address on
// each device once, and only that address is used.
constexpr size_t NOALLOC_SCRATCH_BYTES = 64ull << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
hipError_t g_scratch_err[NOALLOC_MAX_DEVICES] = {};

// With `dev` current: the device address of `scratch` on it (once per device).
void scratch_attach(int dev) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[dev]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    g_scratch_err[dev] = e != hipSuccess ? e : hipErrorInvalidSymbol;
    return;
  }
  g_scratch_ptr[dev] = p;
  g_scratch_err[dev] = hipSuccess;
}

void* scratch_of(int dev) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return g_scratch_ptr[dev];
}

// Bump allocation inside the scratch array for one no-allocation call: a
// per-batch buffer asked for again gets its earlier piece when that is
// large enough, else a new one.
struct NoAllocArena {
  char* base = nullptr;
  size_t cap = 0, top = 0;
  std::vector<std::pair<const DevBuf*, DevBuf>> given;
};

}  // namespace

struct gamma_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  gamma_options opt{};
  std::string last_error;
  bool poisoned = false;
  int n_cu = 256;

  std::vector<DevBuf*> all;

  // graph
  bool has_graph = false;
  uint32_t n = 0;
  int idbits = 1;
  uint64_t live = 0;
  uint64_t arena_cap = 0, arena_top = 0;
  uint32_t label_slots = 1;
  uint32_t n_el = 1, elb = 0;         // edge labels < n_el; row id = v << elb | label
  std::vector<uint64_t> label_count;  // data vertices per label
  DevBuf row_off, row_len, vlabel, label_start, new_of_old, old_of_new, arena, arena_ext;

  // queries
  std::vector<gm::HostQuery> queries;
  uint32_t total_plans = 0;
  uint32_t kmax = 2;
  DevBuf plans, qdev, cand, lab_fstart, fentries, reqs;

  // batch scratch
  DevBuf b_src, b_dst, b_op, b_el, keys, keys_tmp, hist, hist_scan, scan_tmp, keep, ords;
  DevBuf canon_lo, canon_hi, canon_sign, canon_a, canon_b, canon_e, hkeys, hvals, dkeys, dkeys_tmp;
  DevBuf runvals, runscan, touched, run_start, run_end, sizes, r1off, r2_off, r2_len;
  DevBuf seeds, qres, upd_res, tuples, tmeta, tord, ctr, seeds_tmp, gkeys, gkeys_tmp;
  DevBuf tmp64a, tmp64b, tmp32a;
  DevBuf mbox, mflag, idle_bits, idle_rep, seed_open, upd_open;
  DevBuf grp_lead, grp_excl, grp_len, grp_off, grp_lists, seed_grp;  // update-edge grouping
  DevBuf lix, lix_lab, r0_off, r0_len, permtab, qeltab;
  DevBuf vx_src, vx_dst, vx_op, vx_el, vx_del, vx_len, vx_off, vx_mark;  // vertex deletions expanded to edges
  // set during gamma_apply_batch_noalloc: per-batch buffers come from the
  // static scratch array, and nothing may be allocated
  NoAllocArena* na = nullptr;
  std::vector<const DevBuf*> batch_bufs;  // the per-batch buffers
  std::vector<char> h_pageable;           // result staging when the pinned buffer is too small
  uint32_t wall_khz = 100000;
  gamma_tuning tun{};                // search tunables (never change results)
  std::vector<uint32_t> lix_labels;  // labels used by registered queries (label-index slots)

  // host side results
  void* h_pinned = nullptr;
  size_t h_pinned_bytes = 0;
  std::vector<gamma_query_result> hq;
  std::vector<uint32_t> h_canon_lo, h_canon_hi;
  std::vector<uint8_t> h_canon_sign;
  std::vector<uint64_t> h_upd;  // n_canon * 3
  std::vector<uint64_t> h_upd_cnt, h_upd_sum, h_upd_xor;
  std::vector<uint8_t> h_upd_open;
  bool has_result = false;
  uint64_t last_tuples = 0;
  uint32_t last_twidth = 0;
  bool last_has_ord = false;

  hipEvent_t ev[8]{};

  gamma_ctx() {
    DevBuf* list[] = {&row_off, &row_len, &vlabel, &label_start, &new_of_old, &old_of_new, &arena,
                      &arena_ext, &mbox, &mflag, &idle_bits, &idle_rep, &lix, &lix_lab, &r0_off, &r0_len, &permtab, &qeltab,
                      &vx_src, &vx_dst, &vx_op, &vx_el, &vx_del, &vx_len, &vx_off, &vx_mark,
                      &plans, &qdev, &cand, &lab_fstart, &fentries, &reqs, &b_src, &b_dst, &b_op, &b_el,
                      &keys, &keys_tmp, &hist, &hist_scan, &scan_tmp, &keep, &ords, &canon_lo, &canon_e,
                      &canon_hi, &canon_sign, &canon_a, &canon_b, &hkeys, &hvals, &dkeys, &dkeys_tmp,
                      &runvals, &runscan, &touched, &run_start, &run_end, &sizes, &r1off, &r2_off,
                      &r2_len, &seeds, &qres, &upd_res, &tuples, &tmeta, &tord, &ctr, &seeds_tmp, &gkeys, &gkeys_tmp, &tmp64a,
                      &tmp64b, &tmp32a, &seed_open, &upd_open, &grp_lead, &grp_excl, &grp_len, &grp_off,
                      &grp_lists, &seed_grp};
    for (DevBuf* b : list) all.push_back(b);
    const DevBuf* per_batch[] = {&b_src, &b_dst, &b_op, &b_el, &keys, &keys_tmp, &hist, &hist_scan, &scan_tmp,
                                 &keep, &ords, &canon_lo, &canon_hi, &canon_sign, &canon_a, &canon_b, &canon_e,
                                 &hkeys, &hvals, &dkeys, &dkeys_tmp, &runvals, &runscan, &touched, &run_start,
                                 &run_end, &sizes, &r1off, &r2_off, &r2_len, &r0_off, &r0_len, &seeds, &seeds_tmp,
                                 &gkeys, &gkeys_tmp, &qres, &upd_res, &ctr, &tmp64a, &tmp64b, &tmp32a, &mbox,
                                 &mflag, &idle_bits, &idle_rep, &seed_open, &upd_open};
    for (const DevBuf* b : per_batch) batch_bufs.push_back(b);
  }

  bool is_batch_buf(const DevBuf* b) const {
    return std::find(batch_bufs.begin(), batch_bufs.end(), b) != batch_bufs.end();
  }

  void* noalloc_piece(const DevBuf& b, size_t need) {
    for (auto& g : na->given)
      if (g.first == &b && g.second.bytes >= need) return g.second.p;
    const size_t at = (na->top + 255) & ~(size_t)255;
    if (at > na->cap || need > na->cap - at)
      throw StatusError{GAMMA_ENOMEM, "apply_batch_noalloc: the batch needs more than the " +
                                          std::to_string(na->cap >> 20) +
                                          " MiB of the library's no-allocation scratch"};
    na->top = at + need;
    DevBuf d{na->base + at, need};
    for (auto& g : na->given)
      if (g.first == &b) {
        g.second = d;
        return d.p;
      }
    na->given.push_back({&b, d});
    return d.p;
  }

  template <typename T>
  T* ensure(DevBuf& b, size_t count, bool keep_contents = false) {
    size_t need = count * sizeof(T);
    if (need == 0) need = sizeof(T);
    if (na) {
      if (is_batch_buf(&b)) return (T*)noalloc_piece(b, need);
      if (b.bytes >= need) return (T*)b.p;
      throw StatusError{GAMMA_ENOMEM, "apply_batch_noalloc: the context's own device storage would have to grow"};
    }
    if (b.bytes >= need) return (T*)b.p;
    size_t alloc = std::max(need, b.bytes + b.bytes / 2);
    void* p = nullptr;
    if (hipMalloc(&p, alloc) != hipSuccess) {
      (void)hipGetLastError();
      alloc = need;
      if (hipMalloc(&p, alloc) != hipSuccess) {
        (void)hipGetLastError();
        throw StatusError{GAMMA_ENOMEM, "device allocation failed"};
      }
    }
    if (keep_contents && b.p && b.bytes) {
      chk(hipMemcpyAsync(p, b.p, b.bytes, hipMemcpyDeviceToDevice, stream), "copy");
      chk(hipStreamSynchronize(stream), "sync");
    }
    if (b.p) {
      chk(hipStreamSynchronize(stream), "sync");
      chk(hipFree(b.p), "free");
    }
    b.p = p;
    b.bytes = alloc;
    return (T*)p;
  }

  void release(DevBuf& b) {
    if (b.p) {
      (void)hipStreamSynchronize(stream);
      (void)hipFree(b.p);
    }
    b.p = nullptr;
    b.bytes = 0;
  }

  void* pinned(size_t bytes) {
    if (na && h_pinned_bytes < bytes) {
      // no pinned allocation during a no-allocation call: pageable staging
      if (h_pageable.size() < bytes) h_pageable.resize(bytes);
      return h_pageable.data();
    }
    if (h_pinned_bytes < bytes) {
      if (h_pinned) (void)hipHostFree(h_pinned);
      h_pinned = nullptr;
      size_t alloc = std::max(bytes, (size_t)4096);
      if (hipHostMalloc(&h_pinned, alloc, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        h_pinned = nullptr;
        h_pinned_bytes = 0;
        throw StatusError{GAMMA_ENOMEM, "pinned host allocation failed"};
      }
      h_pinned_bytes = alloc;
    }
    return h_pinned;
  }

  GmGraphDev G() {
    GmGraphDev g;
    g.n = n;
    g.idbits = idbits;
    g.row_off = (uint64_t*)row_off.p;
    g.row_len = (uint32_t*)row_len.p;
    g.col = (uint32_t*)arena.p;
    g.ext = (uint32_t*)arena_ext.p;
    g.vlabel = (const uint16_t*)vlabel.p;
    g.label_start = (const uint32_t*)label_start.p;
    g.label_slots = label_slots;
    g.new_of_old = (const uint32_t*)new_of_old.p;
    g.old_of_new = (const uint32_t*)old_of_new.p;
    g.elb = elb;
    g.n_el = n_el;
    return g;
  }
  uint32_t rows() const { return n << elb; }

  void sort_keys(uint64_t* k, uint64_t* tmp, size_t cnt, int bits) {
    if (cnt < 2) return;
    uint32_t* h = ensure<uint32_t>(hist, gm::radix_hist_elems(cnt));
    uint32_t* hs = ensure<uint32_t>(hist_scan, gm::radix_hist_elems(cnt) + 1);
    uint32_t* st = ensure<uint32_t>(scan_tmp, gm::scan_tmp_elems(gm::radix_hist_elems(cnt)));
    gm::radix_sort_u64(k, tmp, cnt, bits, h, hs, st, stream);
  }

  void scan64(const uint64_t* in, uint64_t* out, size_t cnt) {
    uint64_t* t = ensure<uint64_t>(tmp64b, gm::scan_tmp_elems(cnt));
    gm::scan_u64(in, out, cnt, t, stream);
  }
  void scan32(const uint32_t* in, uint32_t* out, size_t cnt) {
    uint32_t* t = ensure<uint32_t>(tmp32a, gm::scan_tmp_elems(cnt));
    gm::scan_u32(in, out, cnt, t, stream);
  }

  void rebuild_filter_tables() {
    std::vector<uint32_t> fs;
    std::vector<GmFilterEntry> fe;
    std::vector<GmReq> rq;
    gm::build_filter_tables(queries, label_slots, fs, fe, rq);
    uint32_t* dfs = ensure<uint32_t>(lab_fstart, fs.size());
    GmFilterEntry* dfe = ensure<GmFilterEntry>(fentries, fe.size());
    GmReq* drq = ensure<GmReq>(reqs, rq.size());
    chk(hipMemcpyAsync(dfs, fs.data(), fs.size() * 4, hipMemcpyHostToDevice, stream), "h2d");
    chk(hipMemcpyAsync(dfe, fe.data(), fe.size() * sizeof(GmFilterEntry), hipMemcpyHostToDevice, stream),
        "h2d");
    chk(hipMemcpyAsync(drq, rq.data(), rq.size() * sizeof(GmReq), hipMemcpyHostToDevice, stream), "h2d");
    chk(hipStreamSynchronize(stream), "sync");
  }

  void upload_plans() {
    std::vector<GmPlan> all_plans;
    std::vector<GmQueryDev> qd;
    std::vector<uint8_t> qel;  // [nq][16][16]
    lix_labels.clear();
    for (auto& q : queries)
      for (uint32_t l : q.labels) lix_labels.push_back(l);
    std::sort(lix_labels.begin(), lix_labels.end());
    lix_labels.erase(std::unique(lix_labels.begin(), lix_labels.end()), lix_labels.end());
    for (auto& q : queries)
      for (auto& p : q.plans)
        for (uint32_t l = 0; l < q.k; ++l)
          p.lslot[l] = (uint32_t)(std::lower_bound(lix_labels.begin(), lix_labels.end(), p.lab[l]) -
                                  lix_labels.begin());
    if (!lix_labels.empty()) {
      uint32_t* dl = ensure<uint32_t>(lix_lab, lix_labels.size());
      chk(hipMemcpyAsync(dl, lix_labels.data(), lix_labels.size() * 4, hipMemcpyHostToDevice, stream), "h2d");
    }
    std::vector<GmPerm> all_perms;
    for (auto& q : queries) {
      GmQueryDev d{};
      d.k = q.k;
      d.plan_base = (uint32_t)all_plans.size();
      d.n_plans = (uint32_t)q.plans.size();
      // a query edge label the graph has no rows for: no match can exist,
      // and the query gets no seeds (its rows would not be addressable)
      uint32_t max_el = 0;
      for (uint32_t e : q.elabels) max_el = std::max(max_el, e);
      if (has_graph && max_el >= n_el) d.n_plans = 0;
      if (q.paused) d.n_plans = 0;  // no seeds, so no search and no results
      qd.push_back(d);
      const size_t t0 = qel.size();
      qel.resize(t0 + GM_MAX_K * GM_MAX_K, 0);
      for (size_t e = 0; e < q.edges.size(); ++e) {
        const uint32_t a = q.edges[e].first, b = q.edges[e].second;
        qel[t0 + a * GM_MAX_K + b] = qel[t0 + b * GM_MAX_K + a] = (uint8_t)q.elabels[e];
      }
      const uint32_t pofs = (uint32_t)all_perms.size();
      const uint32_t cofs = pofs + (uint32_t)q.perms.size();
      for (auto& p : q.plans) {
        GmPlan pp = p;
        pp.perm_base += pofs;
        pp.cperm_base += cofs;
        all_plans.push_back(pp);
      }
      all_perms.insert(all_perms.end(), q.perms.begin(), q.perms.end());
      all_perms.insert(all_perms.end(), q.cperms.begin(), q.cperms.end());
    }
    if (!all_perms.empty()) {
      GmPerm* dperm = ensure<GmPerm>(permtab, all_perms.size());
      chk(hipMemcpyAsync(dperm, all_perms.data(), all_perms.size() * sizeof(GmPerm), hipMemcpyHostToDevice,
                         stream),
          "h2d");
    }
    total_plans = (uint32_t)all_plans.size();
    uint8_t* dqel = ensure<uint8_t>(qeltab, std::max<size_t>(qel.size(), 1));
    if (!qel.empty()) chk(hipMemcpyAsync(dqel, qel.data(), qel.size(), hipMemcpyHostToDevice, stream), "h2d");
    GmPlan* dp = ensure<GmPlan>(plans, std::max<size_t>(all_plans.size(), 1));
    GmQueryDev* dq = ensure<GmQueryDev>(qdev, std::max<size_t>(qd.size(), 1));
    if (!all_plans.empty())
      chk(hipMemcpyAsync(dp, all_plans.data(), all_plans.size() * sizeof(GmPlan), hipMemcpyHostToDevice,
                         stream),
          "h2d");
    if (!qd.empty())
      chk(hipMemcpyAsync(dq, qd.data(), qd.size() * sizeof(GmQueryDev), hipMemcpyHostToDevice, stream),
          "h2d");
    chk(hipStreamSynchronize(stream), "sync");
  }

  // Label index of every row for the current label-index slots.
  void full_label_index() {
    if (!has_graph || lix_labels.empty()) return;
    unsigned long long* L = (unsigned long long*)ensure<uint64_t>(lix, (size_t)rows() * lix_labels.size());
    gm::launch_label_index(G(), nullptr, rows(), (const uint32_t*)lix_lab.p, (uint32_t)lix_labels.size(), L,
                           stream);
    chk(hipGetLastError(), "label index launch");
    chk(hipStreamSynchronize(stream), "sync");
  }

  void touched_label_index(const uint32_t* verts, uint32_t nv) {
    if (lix_labels.empty()) return;
    gm::launch_label_index(G(), verts, nv, (const uint32_t*)lix_lab.p, (uint32_t)lix_labels.size(),
                           (unsigned long long*)lix.p, stream);
  }

  // Candidate table for every query (or one) over all vertices.
  void full_filter(uint32_t only_q) {
    if (!has_graph || queries.empty()) return;
    uint16_t* c = ensure<uint16_t>(cand, (size_t)queries.size() * n, true);
    if (only_q == 0xFFFFFFFFu) {
      gm::fill_u32((uint32_t*)c, 0, ((size_t)queries.size() * n + 1) / 2, stream);
    } else {
      chk(hipMemsetAsync(c + (size_t)only_q * n, 0, (size_t)n * 2, stream), "memset");
    }
    gm::launch_filter(G(), nullptr, n, 0, (const uint32_t*)lab_fstart.p, (const GmFilterEntry*)fentries.p,
                      (const GmReq*)reqs.p, c, only_q, stream);
    chk(hipGetLastError(), "filter launch");
    chk(hipStreamSynchronize(stream), "sync");
  }
};

namespace {

gamma_status fail(gamma_ctx* c, gamma_status s, const std::string& msg) {
  if (c) c->last_error = msg;
  return s;
}

template <typename F>
gamma_status guarded(gamma_ctx* c, F&& f) {
  if (!c) return GAMMA_EINVAL;
  if (c->poisoned) return GAMMA_EDEVICE;
  try {
    return f();
  } catch (const DeviceError& e) {
    c->poisoned = true;
    c->last_error = std::string(e.what) + ": " + hipGetErrorString(e.e);
    return GAMMA_EDEVICE;
  } catch (const StatusError& e) {
    c->last_error = e.msg;
    return e.s;
  } catch (const std::bad_alloc&) {
    c->last_error = "host allocation failed";
    return GAMMA_ENOMEM;
  }
}

// Host copy of a possibly-device input into a device buffer.
template <typename T>
const T* stage_in(gamma_ctx* c, DevBuf& buf, const T* src, size_t count, gamma_mem where) {
  if (where == GAMMA_MEM_DEVICE) return src;
  T* d = c->ensure<T>(buf, count);
  if (count) chk(hipMemcpyAsync(d, src, count * sizeof(T), hipMemcpyHostToDevice, c->stream), "h2d");
  return d;
}

}  // namespace

extern "C" {

uint32_t gamma_version(void) { return 100; }

const char* gamma_status_string(gamma_status s) {
  switch (s) {
    case GAMMA_OK: return "ok";
    case GAMMA_TRUNCATED: return "tuple capacity reached (counts exact)";
    case GAMMA_EINVAL: return "invalid argument";
    case GAMMA_ECONFLICT: return "batch inserts and deletes the same edge";
    case GAMMA_ENOMEM: return "out of memory";
    case GAMMA_EUNSUPPORTED: return "unsupported";
    case GAMMA_ESTATE: return "invalid call order";
    case GAMMA_ETIMEDOUT: return "deadline exceeded";
    case GAMMA_EDEVICE: return "device error";
  }
  return "unknown status";
}

const char* gamma_last_error(const gamma_ctx* ctx) {
  return ctx ? ctx->last_error.c_str() : "null context";
}

gamma_status gamma_create(const gamma_options* opt, gamma_ctx** out) {
  if (!out) return GAMMA_EINVAL;
  *out = nullptr;
  gamma_ctx* c = new (std::nothrow) gamma_ctx();
  if (!c) return GAMMA_ENOMEM;
  if (opt) c->opt = *opt;
  c->device = c->opt.device;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || c->device < 0 || c->device >= ndev) {
    (void)hipGetLastError();
    delete c;
    return GAMMA_EDEVICE;
  }
  if (hipSetDevice(c->device) != hipSuccess) {
    delete c;
    return GAMMA_EDEVICE;
  }
  if (c->opt.stream) {
    c->stream = (hipStream_t)c->opt.stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return GAMMA_EDEVICE;
    }
    c->own_stream = true;
  }
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && cu > 0)
    c->n_cu = cu;
  int wk = 0;
  if (hipDeviceGetAttribute(&wk, hipDeviceAttributeWallClockRate, c->device) == hipSuccess && wk > 0)
    c->wall_khz = (uint32_t)wk;
  for (auto& e : c->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      delete c;
      return GAMMA_EDEVICE;
    }
  scratch_attach(c->device);  // the no-allocation entry point's scratch on this device
  // defaults: as many waves per CU as stay resident with the search
  // kernel's register use (16 for the lean build), few hand-over attempts
  // per idle wave (contending donors cost more than they save, measured on
  // the mid workload), a 10 us poll
  c->tun.waves_per_cu = c->opt.waves_per_cu ? std::min<uint32_t>(c->opt.waves_per_cu, 32)
                                            : std::min<uint32_t>(gm::dfs_resident_waves_per_cu(), 32);
  c->tun.steal = (c->opt.steal_set && !c->opt.steal) ? 2 : 1;
  c->tun.poll_cycles = 24000;  // ~10 us at 2.4 GHz
  c->tun.split_inner = 128;
  c->tun.split_leaf = 512;
  c->tun.query_launch = 1;
  c->tun.handover_gate = 2;
  c->tun.coalesced_search = 2;
  c->tun.group_seeds = 1;
  c->tun.shared_leaf = 2;
  *out = c;
  return GAMMA_OK;
}

gamma_status gamma_destroy(gamma_ctx* c) {
  if (!c) return GAMMA_OK;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (DevBuf* b : c->all)
    if (b->p) (void)hipFree(b->p);
  if (c->h_pinned) (void)hipHostFree(c->h_pinned);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return GAMMA_OK;
}

static gamma_status load_graph_impl(gamma_ctx* c, uint32_t n, uint64_t nnz, const uint64_t* row_ptr,
                             const uint32_t* col, const uint32_t* labels, const uint32_t* elabels, uint32_t n_el,
                             gamma_mem where) {
  return guarded(c, [&]() -> gamma_status {
    if (n == 0 || n >= 0x80000000u || !row_ptr || !labels || (nnz && !col))
      return fail(c, GAMMA_EINVAL, "load_graph: bad sizes or null arrays");
    if (nnz >= 0xFFFFFFFFull) return fail(c, GAMMA_EUNSUPPORTED, "load_graph: nnz must be < 2^32");
    if (n_el == 0 || n_el > GAMMA_MAX_EDGE_LABELS || (!elabels && n_el != 1))
      return fail(c, GAMMA_EINVAL, "load_graph: edge label count must be 1 without labels, 1..256 with them");
    const uint32_t elb = n_el > 1 ? (uint32_t)bits_for(n_el) : 0u;
    const int ib = bits_for(n);
    if (((uint64_t)n << elb) >= 0x80000000ull || 2 * ib + (int)elb + 1 > 64)
      return fail(c, GAMMA_EUNSUPPORTED, "load_graph: n times the edge-label count is too large");
    chk(hipSetDevice(c->device), "set device");
    hipStream_t s = c->stream;
    // stage inputs
    DevBuf in_rp, in_col, in_lab, in_el;
    struct Tmp {
      gamma_ctx* c;
      DevBuf* b[4];
      ~Tmp() {
        for (DevBuf* x : b) c->release(*x);
      }
    } tmp{c, {&in_rp, &in_col, &in_lab, &in_el}};
    const uint64_t* d_rp = stage_in<uint64_t>(c, in_rp, row_ptr, (size_t)n + 1, where);
    const uint32_t* d_col = nnz ? stage_in<uint32_t>(c, in_col, col, nnz, where) : nullptr;
    const uint32_t* d_lab = stage_in<uint32_t>(c, in_lab, labels, n, where);
    const uint32_t* d_el = (elabels && nnz) ? stage_in<uint32_t>(c, in_el, elabels, nnz, where) : nullptr;
    uint32_t* ctrw = (uint32_t*)c->ensure<GmCounters>(c->ctr, 1);
    gm::fill_u32(ctrw, 0, sizeof(GmCounters) / 4, s);
    uint32_t* dummy_col = nullptr;
    if (!d_col) {
      dummy_col = c->ensure<uint32_t>(c->tmp32a, 1);
      d_col = dummy_col;
    }
    gm::launch_validate_csr(d_rp, d_col, d_lab, d_el, n_el, n, nnz, ctrw, s);
    chk(hipGetLastError(), "validate launch");
    uint32_t err = 0;
    chk(hipMemcpyAsync(&err, ctrw, 4, hipMemcpyDeviceToHost, s), "d2h");
    chk(hipStreamSynchronize(s), "sync");
    if (err) return fail(c, GAMMA_EINVAL, "load_graph: malformed CSR or labels (error bits " +
                                              std::to_string(err) + ")");

    // new graph buffers (built aside, swapped in at the end)
    gamma_ctx& C = *c;
    DevBuf n_row_off, n_row_len, n_vlabel, n_label_start, n_n2o, n_o2n, n_arena, n_ext;
    const uint32_t rows = n << elb;
    {
      uint64_t* keys = C.ensure<uint64_t>(C.keys, n);
      uint64_t* kt = C.ensure<uint64_t>(C.keys_tmp, n);
      gm::launch_relabel_keys(d_lab, n, keys, s);
      C.sort_keys(keys, kt, n, 48);
      uint32_t* n2o = C.ensure<uint32_t>(n_n2o, n);
      uint32_t* o2n = C.ensure<uint32_t>(n_o2n, n);
      uint16_t* vl = C.ensure<uint16_t>(n_vlabel, n);
      gm::launch_relabel_apply(keys, n, n2o, o2n, vl, s);
      uint16_t maxlab = 0;
      chk(hipMemcpyAsync(&maxlab, vl + (n - 1), 2, hipMemcpyDeviceToHost, s), "d2h");
      chk(hipStreamSynchronize(s), "sync");
      uint32_t slots = (uint32_t)maxlab + 1;
      uint32_t* ls = C.ensure<uint32_t>(n_label_start, slots + 1);
      gm::launch_label_start(vl, n, slots, ls, s);
      std::vector<uint32_t> hls(slots + 1);
      chk(hipMemcpyAsync(hls.data(), ls, (slots + 1) * 4, hipMemcpyDeviceToHost, s), "d2h");
      chk(hipStreamSynchronize(s), "sync");
      C.label_slots = slots;
      C.label_count.assign(slots, 0);
      for (uint32_t l = 0; l < slots; ++l) C.label_count[l] = hls[l + 1] - hls[l];
      // rows in internal ids (with edge labels, rows (v << elb) | label:
      // their lengths come from the sorted entry keys)
      uint64_t* deg = C.ensure<uint64_t>(C.tmp64a, (size_t)rows + 1);
      uint64_t* offs = C.ensure<uint64_t>(C.sizes, (size_t)rows + 1);
      uint64_t* ro = C.ensure<uint64_t>(n_row_off, rows);
      uint32_t* rl = C.ensure<uint32_t>(n_row_len, rows);
      uint64_t cap = nnz + std::max<uint64_t>(nnz / 2, 1u << 20);
      uint32_t* ar = C.ensure<uint32_t>(n_arena, cap);
      uint32_t* ax = C.ensure<uint32_t>(n_ext, cap);
      if (elb == 0) gm::launch_deg_mapped(d_rp, nullptr, n2o, n, deg, s);
      if (nnz) {
        uint64_t* ek = C.ensure<uint64_t>(C.keys, nnz);
        uint64_t* et = C.ensure<uint64_t>(C.keys_tmp, nnz);
        gm::launch_csr_keys(nullptr, nullptr, d_rp, d_col, n2o, n, ib, nullptr, ek, s, d_el, elb);
        C.sort_keys(ek, et, nnz, 2 * ib + (int)elb);
        if (elb) {
          gm::fill_u64(deg, 0, rows, s);
          gm::launch_row_hist(ek, nnz, ib, deg, s);
        }
        gm::launch_csr_extract(ek, nnz, (1ull << ib) - 1, ar, s);
        gm::launch_gather_ext(ar, o2n, nnz, ax, s);
      } else if (elb) {
        gm::fill_u64(deg, 0, rows, s);
      }
      C.scan64(deg, offs, rows);
      gm::launch_rows_from_scan(offs, deg, rows, 0, ro, rl, s);
      chk(hipGetLastError(), "load launch");
      chk(hipStreamSynchronize(s), "sync");
      // the load-time sort buffers are sized by nnz; batches need far less
      C.release(C.keys);
      C.release(C.keys_tmp);
      C.arena_cap = cap;
      C.arena_top = nnz;
    }
    // swap in
    auto swap_in = [&](DevBuf& dst, DevBuf& src) {
      C.release(dst);
      dst = src;
      src = DevBuf{};
    };
    swap_in(C.row_off, n_row_off);
    swap_in(C.row_len, n_row_len);
    swap_in(C.vlabel, n_vlabel);
    swap_in(C.label_start, n_label_start);
    swap_in(C.new_of_old, n_n2o);
    swap_in(C.old_of_new, n_o2n);
    swap_in(C.arena, n_arena);
    swap_in(C.arena_ext, n_ext);
    C.n = n;
    C.idbits = ib;
    C.n_el = n_el;
    C.elb = elb;
    C.live = nnz;
    C.has_graph = true;
    C.has_result = false;
    // queries: re-plan (label frequencies changed), re-filter
    if (!C.queries.empty()) {
      for (uint32_t qi = 0; qi < C.queries.size(); ++qi) gm::plan_query(C.queries[qi], qi, C.label_count);
      C.upload_plans();
      C.rebuild_filter_tables();
      C.release(C.cand);
      C.full_filter(0xFFFFFFFFu);
      C.release(C.lix);
      C.full_label_index();
    }
    return GAMMA_OK;
  });
}

gamma_status gamma_load_graph(gamma_ctx* c, uint32_t n, uint64_t nnz, const uint64_t* row_ptr,
                              const uint32_t* col, const uint32_t* labels, gamma_mem where) {
  return load_graph_impl(c, n, nnz, row_ptr, col, labels, nullptr, 1, where);
}

gamma_status gamma_load_graph_el(gamma_ctx* c, uint32_t n, uint64_t nnz, const uint64_t* row_ptr,
                                 const uint32_t* col, const uint32_t* labels, const uint32_t* elabels,
                                 uint32_t n_elabels, gamma_mem where) {
  return load_graph_impl(c, n, nnz, row_ptr, col, labels, elabels, n_elabels, where);
}

gamma_status gamma_register_query_el(gamma_ctx* c, uint32_t k, const uint32_t* qlabels, uint32_t m,
                                     const uint32_t* qedges, const uint32_t* qelabels, uint32_t* out_qid) {
  return guarded(c, [&]() -> gamma_status {
    std::string msg;
    int st = gm::validate_query(k, qlabels, m, qedges, &msg);
    if (st != GAMMA_OK) return fail(c, (gamma_status)st, "register_query: " + msg);
    for (uint32_t e = 0; qelabels && e < m; ++e)
      if (qelabels[e] >= GAMMA_MAX_EDGE_LABELS) return fail(c, GAMMA_EINVAL, "register_query: edge label >= 256");
    if (c->queries.size() >= 4096) return fail(c, GAMMA_EUNSUPPORTED, "register_query: too many queries");
    chk(hipSetDevice(c->device), "set device");
    gm::HostQuery q;
    q.k = k;
    q.labels.assign(qlabels, qlabels + k);
    for (uint32_t e = 0; e < m; ++e) q.edges.push_back({qedges[2 * e], qedges[2 * e + 1]});
    q.elabels.assign(m, 0);
    if (qelabels) q.elabels.assign(qelabels, qelabels + m);
    uint32_t qi = (uint32_t)c->queries.size();
    gm::plan_query(q, qi, c->label_count);
    c->queries.push_back(q);
    try {
      c->upload_plans();
      c->kmax = std::max(c->kmax, k);
      if (c->has_graph) {
        c->rebuild_filter_tables();
        c->full_filter(qi);
        c->full_label_index();
      }
    } catch (const StatusError&) {
      c->queries.pop_back();
      throw;
    }
    if (out_qid) *out_qid = qi;
    return GAMMA_OK;
  });
}

gamma_status gamma_register_query(gamma_ctx* c, uint32_t k, const uint32_t* qlabels, uint32_t m,
                                  const uint32_t* qedges, uint32_t* out_qid) {
  return gamma_register_query_el(c, k, qlabels, m, qedges, nullptr, out_qid);
}

namespace {

// Move every row into a fresh, larger arena (rows contiguous, no garbage).
void compact_arena(gamma_ctx* c, uint64_t need) {
  hipStream_t s = c->stream;
  const uint32_t n = c->rows();  // every row, one per (vertex, edge label)
  uint64_t cap = std::max<uint64_t>(c->arena_cap, 2 * (c->live + need) + (1u << 20));
  DevBuf na, nx;
  uint32_t* dst = c->ensure<uint32_t>(na, cap);
  uint32_t* dstx = c->ensure<uint32_t>(nx, cap);
  uint64_t* deg = c->ensure<uint64_t>(c->tmp64a, (size_t)n + 1);
  gm::launch_deg_mapped(nullptr, (const uint32_t*)c->row_len.p, nullptr, n, deg, s);
  uint64_t* offs = c->ensure<uint64_t>(c->sizes, (size_t)n + 1);
  c->scan64(deg, offs, n);
  gm::launch_copy_rows((const uint64_t*)c->row_off.p, (const uint32_t*)c->row_len.p,
                       (const uint32_t*)c->arena.p, offs, dst, n, s);
  gm::launch_copy_rows((const uint64_t*)c->row_off.p, (const uint32_t*)c->row_len.p,
                       (const uint32_t*)c->arena_ext.p, offs, dstx, n, s);
  gm::launch_rows_from_scan(offs, deg, n, 0, (uint64_t*)c->row_off.p, nullptr, s);
  chk(hipGetLastError(), "compact launch");
  chk(hipStreamSynchronize(s), "sync");
  c->release(c->arena);
  c->release(c->arena_ext);
  c->arena = na;
  c->arena_ext = nx;
  c->arena_cap = cap;
  c->arena_top = c->live;
}

}  // namespace

gamma_status gamma_apply_batch_el(gamma_ctx* c, uint32_t n_upd, const uint32_t* src, const uint32_t* dst,
                                  const uint8_t* op, const uint32_t* elab, gamma_mem where, uint32_t flags,
                                  gamma_batch_result* out) {
  return guarded(c, [&]() -> gamma_status {
    if (!out) return fail(c, GAMMA_EINVAL, "apply_batch: null result");
    if (!c->has_graph) return fail(c, GAMMA_ESTATE, "apply_batch: no graph loaded");
    if (n_upd > (1u << 20)) return fail(c, GAMMA_EINVAL, "apply_batch: more than 2^20 updates");
    if (n_upd && (!src || !dst || !op)) return fail(c, GAMMA_EINVAL, "apply_batch: null update arrays");
    if ((flags & GAMMA_F_TUPLES) && c->opt.tuple_capacity == 0)
      return fail(c, GAMMA_EINVAL, "apply_batch: TUPLES requested but tuple_capacity is 0");
    chk(hipSetDevice(c->device), "set device");
    gamma_ctx& C = *c;
    hipStream_t s = C.stream;
    C.has_result = false;
    const uint32_t nq = (uint32_t)C.queries.size();
    const uint32_t n = C.n;
    const int eb = C.idbits;
    const int ib = C.idbits;
    chk(hipEventRecord(C.ev[0], s), "event");

    // ---------------------------------------------------------- canonicalise
    const uint32_t* d_src = stage_in<uint32_t>(c, C.b_src, src, n_upd, where);
    const uint32_t* d_dst = stage_in<uint32_t>(c, C.b_dst, dst, n_upd, where);
    const uint8_t* d_op = stage_in<uint8_t>(c, C.b_op, op, n_upd, where);
    const uint32_t* d_el = (elab && n_upd) ? stage_in<uint32_t>(c, C.b_el, elab, n_upd, where) : nullptr;
    const int elb = (int)C.elb;
    GmCounters* ctr = C.ensure<GmCounters>(C.ctr, 1);
    gm::fill_u32((uint32_t*)ctr, 0, sizeof(GmCounters) / 4, s);
    const size_t nu = std::max<uint32_t>(n_upd, 1);
    uint64_t* keys = C.ensure<uint64_t>(C.keys, nu);
    uint64_t* kt = C.ensure<uint64_t>(C.keys_tmp, std::max<size_t>(2 * nu, 2));
    uint32_t* keep = C.ensure<uint32_t>(C.keep, nu);
    uint32_t* ords = C.ensure<uint32_t>(C.ords, nu + 1);
    GmGraphDev G = C.G();
    gm::launch_canon_keys(d_src, d_dst, d_op, d_el, n_upd, n, eb, C.elb, C.n_el, keys, ctr, s);
    C.sort_keys(keys, kt, n_upd, 2 * eb + elb + 1);
    gm::launch_canon_classify(keys, n_upd, eb, G, keep, ctr, s);
    C.scan32(keep, ords, n_upd);
    uint32_t hcap = 64;
    while (hcap < 2 * nu) hcap <<= 1;
    GmBatchHash H;
    H.keys = C.ensure<uint64_t>(C.hkeys, hcap);
    H.vals = C.ensure<uint32_t>(C.hvals, hcap);
    H.mask = hcap - 1;
    gm::fill_u64(H.keys, GM_EMPTY64, hcap, s);
    uint32_t* clo = C.ensure<uint32_t>(C.canon_lo, nu);
    uint32_t* chi = C.ensure<uint32_t>(C.canon_hi, nu);
    uint8_t* csg = C.ensure<uint8_t>(C.canon_sign, nu);
    uint32_t* ca = C.ensure<uint32_t>(C.canon_a, nu);
    uint32_t* cb = C.ensure<uint32_t>(C.canon_b, nu);
    const size_t N2 = 2 * nu;  // directed entries, padded
    uint64_t* dk = C.ensure<uint64_t>(C.dkeys, N2);
    uint64_t* dkt = C.ensure<uint64_t>(C.dkeys_tmp, N2);
    uint32_t* cel = elb ? C.ensure<uint32_t>(C.canon_e, nu) : nullptr;
    gm::launch_canon_emit(keys, keep, ords, n_upd, eb, G, clo, chi, csg, ca, cb, cel, H, dk, s);
    // the canonical count decides the directed sort length: one sync here,
    // before anything is mutated, also reports validation errors
    struct {
      uint32_t n_canon;
      uint32_t pad;
    } h1{};
    GmCounters hc{};
    chk(hipMemcpyAsync(&h1.n_canon, ords + n_upd, 4, hipMemcpyDeviceToHost, s), "d2h");
    chk(hipMemcpyAsync(&hc, ctr, sizeof(GmCounters), hipMemcpyDeviceToHost, s), "d2h");
    chk(hipStreamSynchronize(s), "sync");
    chk(hipGetLastError(), "canon launch");
    if (hc.err & (GM_ERR_RANGE | GM_ERR_SELFLOOP))
      return fail(c, GAMMA_EINVAL, "apply_batch: vertex id or edge label out of range, or self loop");
    if (hc.err & GM_ERR_RELABEL)
      return fail(c, GAMMA_EINVAL, "apply_batch: an inserted pair is present under another edge label");
    if (hc.err & GM_ERR_CONFLICT)
      return fail(c, GAMMA_ECONFLICT, "apply_batch: an edge is both inserted and deleted");
    const uint32_t n_canon = n_upd ? h1.n_canon : 0;
    const uint32_t N = 2 * n_canon;
    C.sort_keys(dk, dkt, N, 2 * ib + elb + 1);
    uint64_t* rv = C.ensure<uint64_t>(C.runvals, std::max<uint32_t>(N, 1));
    uint64_t* rsc = C.ensure<uint64_t>(C.runscan, (size_t)N + 1);
    gm::launch_runs_flags(dk, N, ib, rv, s);
    C.scan64(rv, rsc, N);
    uint32_t* tch = C.ensure<uint32_t>(C.touched, std::max<uint32_t>(N, 1));
    uint32_t* rs_ = C.ensure<uint32_t>(C.run_start, std::max<uint32_t>(N, 1));
    uint32_t* re_ = C.ensure<uint32_t>(C.run_end, std::max<uint32_t>(N, 1));
    gm::launch_runs_fill(dk, rsc, N, ib, tch, rs_, re_, s);
    uint64_t hrun = 0;
    chk(hipMemcpyAsync(&hrun, rsc + N, 8, hipMemcpyDeviceToHost, s), "d2h");
    chk(hipStreamSynchronize(s), "sync");
    const uint32_t n_touched = (uint32_t)hrun;
    const uint32_t n_ins_dir = (uint32_t)(hrun >> 32);
    const uint32_t n_insert = n_ins_dir / 2;
    const uint32_t n_delete = n_canon - n_insert;
    uint64_t* sz = C.ensure<uint64_t>(C.sizes, std::max<uint32_t>(n_touched, 1));
    uint64_t* r1 = C.ensure<uint64_t>(C.r1off, (size_t)n_touched + 1);
    gm::launch_touched_sizes(tch, rs_, re_, rsc, n_touched, G, sz, s);
    C.scan64(sz, r1, n_touched);
    uint64_t r1_total = 0;
    chk(hipMemcpyAsync(&r1_total, r1 + n_touched, 8, hipMemcpyDeviceToHost, s), "d2h");
    chk(hipStreamSynchronize(s), "sync");
    chk(hipGetLastError(), "runs launch");
    chk(hipEventRecord(C.ev[1], s), "event");

    // ---------------------------------------------------------- delta-merge
    const uint64_t r2_total = r1_total - 2ull * n_delete;
    if (C.arena_top + r1_total + r2_total > C.arena_cap) {
      if (C.na)
        return fail(c, GAMMA_ENOMEM, "apply_batch_noalloc: the graph's arena is full (a gamma_apply_batch call "
                                     "compacts it)");
      compact_arena(c, r1_total + r2_total);
      G = C.G();
    }
    // every buffer the rest of the batch needs is sized here, before the
    // graph is touched, so that running out of memory leaves it unchanged
    const uint64_t base1 = C.arena_top, base2 = base1 + r1_total;
    uint64_t* r2o = C.ensure<uint64_t>(C.r2_off, std::max<uint32_t>(n_touched, 1));
    uint32_t* r2l = C.ensure<uint32_t>(C.r2_len, std::max<uint32_t>(n_touched, 1));
    uint64_t* r0o = C.ensure<uint64_t>(C.r0_off, std::max<uint32_t>(n_touched, 1));
    uint32_t* r0l = C.ensure<uint32_t>(C.r0_len, std::max<uint32_t>(n_touched, 1));
    const uint64_t seed_cap = std::max<uint64_t>((uint64_t)n_canon * C.total_plans, 1);
    GmSeed* sd = C.ensure<GmSeed>(C.seeds, seed_cap);
    // per query: (count, sum, xor) per sign, then the number of its seeds
    // whose search did not finish
    const size_t qres_n = std::max<size_t>((size_t)nq * 7, 7);
    unsigned long long* qres = C.ensure<unsigned long long>(C.qres, qres_n);
    unsigned long long* upd = nullptr;
    // per-seed completion, tracked with per-update results and under a deadline
    const bool track = (flags & GAMMA_F_PER_UPDATE) || C.opt.deadline_ms;
    uint32_t* sopen = track ? C.ensure<uint32_t>(C.seed_open, seed_cap) : nullptr;
    uint8_t* uopen = nullptr;
    const size_t uopen_words = ((size_t)n_canon + 3) / 4 + 1;
    if (flags & GAMMA_F_PER_UPDATE) {
      upd = C.ensure<unsigned long long>(C.upd_res, std::max<size_t>((size_t)n_canon * 3, 3));
      uopen = (uint8_t*)C.ensure<uint32_t>(C.upd_open, uopen_words);
    }
    const uint32_t wpc = C.tun.waves_per_cu;
    const unsigned blocks = (unsigned)std::max<uint64_t>(1, (uint64_t)C.n_cu * wpc / gm::dfs_waves_per_block());
    const uint32_t slots = gm::dfs_slots(blocks);
    uint32_t* d_mbox = C.ensure<uint32_t>(C.mbox, (size_t)slots * 32);
    uint32_t* d_mflag = C.ensure<uint32_t>(C.mflag, slots);
    unsigned long long* d_idle_bits = (unsigned long long*)C.ensure<uint64_t>(C.idle_bits, (slots + 63) / 64);
    uint32_t* d_idle_rep = C.ensure<uint32_t>(C.idle_rep, 256);
    G = C.G();
    gm::launch_merge(dk, rsc, tch, rs_, re_, r1, n_touched, r1_total, base1, base2, ib, G, s);
    gm::launch_rows_save(tch, n_touched, G, r0o, r0l, s);
    gm::launch_rows_set(tch, rs_, re_, rsc, r1, n_touched, base1, base2, G, r2o, r2l, s);
    C.touched_label_index(tch, n_touched);
    C.arena_top += r1_total + r2_total;
    chk(hipEventRecord(C.ev[2], s), "event");

    // ---------------------------------------------------------- filter refresh (G u I)
    if (nq)
      gm::launch_filter(G, tch, n_touched, 1, (const uint32_t*)C.lab_fstart.p,
                        (const GmFilterEntry*)C.fentries.p, (const GmReq*)C.reqs.p,
                        (uint16_t*)C.cand.p, 0xFFFFFFFFu, s);
    chk(hipEventRecord(C.ev[3], s), "event");

    // ---------------------------------------------------------- seeds
    // (one launch per query: each query's seeds are generated right before
    // its own search launch, so that time falls in the search phase)
    const bool per_query = C.tun.query_launch == 2 && nq > 1;
    const uint32_t* grp_seed = nullptr;  // update-edge grouping, when built
    const GmGroupList* grp_lists = nullptr;
    uint32_t n_groups = 0;
    gm::launch_seed_window(ctr, s);
    if (nq && !per_query) {
      gm::launch_seeds(ca, cb, csg, cel, n_canon, (const GmQueryDev*)C.qdev.p, nq, (const GmPlan*)C.plans.p,
                       (const uint16_t*)C.cand.p, n, sd, seed_cap, ctr, 0xFFFFFFFFu,
                       C.tun.coalesced_search - 1, s);
      if (C.tun.group_seeds == 2 && !C.na) {  // (a tunable: off in a no-allocation call)
        // update-edge grouping: a stable sort of the seeds by their first
        // data vertex (keys: position << ibr | a, ibr = ib rounded up to the
        // sort's 8-bit digits so that no digit mixes in position bits),
        // then a gather
        unsigned long long hn = 0;
        chk(hipMemcpyAsync(&hn, &ctr->n_seeds, 8, hipMemcpyDeviceToHost, s), "d2h");
        chk(hipStreamSynchronize(s), "sync");
        const uint64_t ns = std::min<uint64_t>(hn, seed_cap);
        const int ibr = (ib + 7) & ~7;
        if (ns > 1 && ns < (1ull << (64 - ibr))) {
          uint64_t* gk = C.ensure<uint64_t>(C.gkeys, ns);
          uint64_t* gt = C.ensure<uint64_t>(C.gkeys_tmp, ns);
          GmSeed* so = C.ensure<GmSeed>(C.seeds_tmp, ns);
          gm::launch_seed_keys(sd, ns, ibr, gk, s);
          C.sort_keys(gk, gt, ns, ibr);
          gm::launch_seed_gather(sd, gk, ns, ibr, so, s);
          chk(hipMemcpyAsync(sd, so, ns * sizeof(GmSeed), hipMemcpyDeviceToDevice, s), "copy");
        }
      }
      if (C.tun.group_seeds == 3 && !C.na) {
        // update-edge grouping (Alg. 1 runs its loop over update edges; seeds
        // that map the same directed query edge (x, y) with x onto the same
        // data vertex a share a's candidates for level 2): the seeds are
        // sorted by (query, directed query edge, a), and every group of two
        // or more whose level 2 has a list from a gets that list built once,
        // filtered by the candidate table, in arena space past the batch's
        // rows; its seeds then drive level 2 from it.  Skipped when the
        // arena lacks the room (a tunable: results are the same either way).
        unsigned long long hn = 0;
        chk(hipMemcpyAsync(&hn, &ctr->n_seeds, 8, hipMemcpyDeviceToHost, s), "d2h");
        chk(hipStreamSynchronize(s), "sync");
        const uint64_t ns = std::min<uint64_t>(hn, seed_cap);
        const int pb = bits_for(ns);
        if (ns > 1 && 16 + ib + pb <= 64) {
          uint64_t* gk = C.ensure<uint64_t>(C.gkeys, ns);
          uint64_t* gt = C.ensure<uint64_t>(C.gkeys_tmp, ns);
          GmSeed* so = C.ensure<GmSeed>(C.seeds_tmp, ns);
          gm::launch_group_keys(sd, ns, ib, pb, gk, s);
          C.sort_keys(gk, gt, ns, 16 + ib + pb);
          gm::launch_group_gather(sd, gk, ns, pb, so, s);
          chk(hipMemcpyAsync(sd, so, ns * sizeof(GmSeed), hipMemcpyDeviceToDevice, s), "copy");
          uint32_t* lead = C.ensure<uint32_t>(C.grp_lead, ns);
          uint32_t* excl = C.ensure<uint32_t>(C.grp_excl, ns + 1);
          gm::launch_group_lead(gk, ns, pb, lead, s);
          C.scan32(lead, excl, ns);
          uint32_t ng = 0;
          chk(hipMemcpyAsync(&ng, excl + ns, 4, hipMemcpyDeviceToHost, s), "d2h");
          chk(hipStreamSynchronize(s), "sync");
          unsigned long long* glen = (unsigned long long*)C.ensure<uint64_t>(C.grp_len, std::max<uint32_t>(ng, 1));
          unsigned long long* goff = (unsigned long long*)C.ensure<uint64_t>(C.grp_off, (size_t)ng + 1);
          gm::launch_group_len(sd, excl, lead, ns, (const GmPlan*)C.plans.p, (const GmQueryDev*)C.qdev.p, G,
                               (const unsigned long long*)C.lix.p, (uint32_t)C.lix_labels.size(),
                               (const uint8_t*)C.qeltab.p, glen, s);
          C.scan64((const uint64_t*)glen, (uint64_t*)goff, ng);
          uint64_t gtotal = 0;
          chk(hipMemcpyAsync(&gtotal, goff + ng, 8, hipMemcpyDeviceToHost, s), "d2h");
          chk(hipStreamSynchronize(s), "sync");
          if (C.arena_top + gtotal <= C.arena_cap) {
            GmGroupList* lists = C.ensure<GmGroupList>(C.grp_lists, std::max<uint32_t>(ng, 1));
            uint32_t* sg = C.ensure<uint32_t>(C.seed_grp, ns);
            gm::launch_group_fill(sd, excl, lead, ns, (const GmPlan*)C.plans.p, (const GmQueryDev*)C.qdev.p, G,
                                  (const unsigned long long*)C.lix.p, (uint32_t)C.lix_labels.size(),
                                  (const uint8_t*)C.qeltab.p, (const uint16_t*)C.cand.p,
                                  C.tun.coalesced_search - 1, glen, goff, C.arena_top, lists, s);
            gm::launch_group_assign(excl, lead, ns, sg, s);
            grp_seed = sg;
            grp_lists = lists;
            n_groups = ng;
          }
        }
      }
    }
    chk(hipEventRecord(C.ev[4], s), "event");

    // ---------------------------------------------------------- search
    gm::fill_u64((uint64_t*)qres, 0, qres_n, s);
    if (upd) gm::fill_u64((uint64_t*)upd, 0, (size_t)n_canon * 3, s);
    if (sopen) gm::fill_u32(sopen, 0xFFFFFFFFu, seed_cap, s);
    const uint32_t tw = C.kmax;
    uint64_t tcap = 0;
    if (flags & GAMMA_F_TUPLES) {
      tcap = C.opt.tuple_capacity;
      C.ensure<uint32_t>(C.tuples, tcap * tw);
      C.ensure<uint32_t>(C.tmeta, tcap);
      if (flags & GAMMA_F_SEED_ATTR) C.ensure<uint32_t>(C.tord, tcap);
    }
    if (nq && n_canon) {
      GmDfsParams P{};  // every field defined (pointers the kernel tests stay null unless set)
      P.G = G;
      P.lix = (const unsigned long long*)C.lix.p;
      P.lix_slots = (uint32_t)C.lix_labels.size();
      P.plans = (const GmPlan*)C.plans.p;
      P.queries = (const GmQueryDev*)C.qdev.p;
      P.cand = (const uint16_t*)C.cand.p;
      P.seeds = sd;
      P.H = H;
      P.ctr = ctr;
      P.flags = flags & (GM_F_HASH | GM_F_TUPLES | GM_F_SEED_ATTR | GM_F_PER_UPDATE);
      P.twidth = tw;
      P.qres = qres;
      P.tuples = (uint32_t*)C.tuples.p;
      P.tmeta = (uint32_t*)C.tmeta.p;
      P.tord = (uint32_t*)C.tord.p;
      P.tcap = tcap;
      P.upd_res = upd;
      P.mbox = d_mbox;
      P.mflag = d_mflag;
      P.idle_bits = d_idle_bits;
      P.idle_rep = d_idle_rep;
      P.n_slots = slots;
      P.donate = C.tun.steal == 1 ? 1u : 0u;
      P.deadline_ticks = (uint64_t)C.opt.deadline_ms * C.wall_khz;
      P.poll_cycles = C.tun.poll_cycles;
      P.split_inner = C.tun.split_inner;
      P.split_leaf = C.tun.split_leaf;
      P.gate = C.tun.handover_gate;
      P.shared_leaf = C.tun.shared_leaf >= 2 ? 1u : 0u;
      P.reenter = C.tun.shared_leaf == 2 ? 1u : 0u;
      P.perms = (const GmPerm*)C.permtab.p;
      // plans permute matches only when some query (or core) has symmetries;
      // without them coalescing changes nothing and the lean search applies
      uint32_t coal = C.tun.coalesced_search - 1;
      bool permutes = false;
      for (const auto& hq : C.queries)
        for (const auto& pl : hq.plans) permutes = permutes || pl.n_perm >= 2 || (coal >= 2 && pl.n_cperm >= 2);
      P.coalesce = permutes ? coal : 0u;
      P.qel = (const uint8_t*)C.qeltab.p;
      P.seed_open = sopen;
      P.seed_group = grp_seed;
      P.group_list = grp_lists;
      for (uint32_t qi = 0; qi < (per_query ? nq : 1u); ++qi) {
        if (per_query) {
          if (C.queries[qi].paused) continue;
          if (qi) gm::launch_seed_window(ctr, s);
          gm::launch_seeds(ca, cb, csg, cel, n_canon, (const GmQueryDev*)C.qdev.p, nq, (const GmPlan*)C.plans.p,
                           (const uint16_t*)C.cand.p, n, sd, seed_cap, ctr, qi,
                           C.tun.coalesced_search - 1, s);
        }
        gm::fill_u32(P.mflag, 0, slots, s);
        gm::fill_u64((uint64_t*)P.idle_bits, 0, (slots + 63) / 64, s);
        gm::fill_u32(P.idle_rep, 0, 256, s);
        gm::launch_pending_init(ctr, s);
        gm::launch_dfs(P, blocks, s);
      }
    }
    chk(hipEventRecord(C.ev[5], s), "event");
    if (uopen) gm::fill_u32((uint32_t*)uopen, 0, uopen_words, s);
    if (sopen && nq && n_canon) gm::launch_upd_open(sd, ctr, seed_cap, sopen, uopen, qres + (size_t)nq * 6, s);

    // ---------------------------------------------------------- commit G', refresh filter on G'
    // a dry run (or a search past its deadline) puts the saved rows back
    const bool dry = (flags & GAMMA_F_DRY_RUN) != 0;
    gm::launch_rows_finish(tch, r2o, r2l, r0o, r0l, n_touched, G, ctr, dry ? 1u : 0u, s);
    C.touched_label_index(tch, n_touched);
    if (nq)
      gm::launch_filter(G, tch, n_touched, 1, (const uint32_t*)C.lab_fstart.p,
                        (const GmFilterEntry*)C.fentries.p, (const GmReq*)C.reqs.p,
                        (uint16_t*)C.cand.p, 0xFFFFFFFFu, s);
    chk(hipEventRecord(C.ev[6], s), "event");

    // ---------------------------------------------------------- results to host
    size_t hbytes = qres_n * 8 + sizeof(GmCounters);
    if (flags & GAMMA_F_PER_UPDATE) hbytes += (size_t)n_canon * 25;
    if (flags & GAMMA_F_CANONICAL) hbytes += (size_t)n_canon * 9;
    char* hp = (char*)C.pinned(hbytes);
    uint64_t* h_qres = (uint64_t*)hp;
    GmCounters* h_ctr = (GmCounters*)(hp + qres_n * 8);
    char* tail = hp + qres_n * 8 + sizeof(GmCounters);
    chk(hipMemcpyAsync(h_qres, qres, qres_n * 8, hipMemcpyDeviceToHost, s), "d2h");
    chk(hipMemcpyAsync(h_ctr, ctr, sizeof(GmCounters), hipMemcpyDeviceToHost, s), "d2h");
    uint64_t* h_upd = nullptr;
    if ((flags & GAMMA_F_PER_UPDATE) && n_canon) {
      h_upd = (uint64_t*)tail;
      chk(hipMemcpyAsync(h_upd, upd, (size_t)n_canon * 24, hipMemcpyDeviceToHost, s), "d2h");
      tail += (size_t)n_canon * 24;
    }
    uint8_t* h_uopen = nullptr;
    if ((flags & GAMMA_F_PER_UPDATE) && n_canon) {
      h_uopen = (uint8_t*)tail;
      chk(hipMemcpyAsync(h_uopen, uopen, n_canon, hipMemcpyDeviceToHost, s), "d2h");
      tail += n_canon;
    }
    uint32_t* h_clo = nullptr;
    if ((flags & GAMMA_F_CANONICAL) && n_canon) {
      h_clo = (uint32_t*)tail;
      chk(hipMemcpyAsync(h_clo, clo, (size_t)n_canon * 4, hipMemcpyDeviceToHost, s), "d2h");
      chk(hipMemcpyAsync(h_clo + n_canon, chi, (size_t)n_canon * 4, hipMemcpyDeviceToHost, s), "d2h");
      chk(hipMemcpyAsync(h_clo + 2 * (size_t)n_canon, csg, n_canon, hipMemcpyDeviceToHost, s), "d2h");
    }
    chk(hipEventRecord(C.ev[7], s), "event");
    chk(hipStreamSynchronize(s), "sync");
    chk(hipGetLastError(), "batch launch");

    // ---------------------------------------------------------- fill the result
    C.hq.assign(nq, gamma_query_result{});
    for (uint32_t q = 0; q < nq; ++q) {
      gamma_query_result& r = C.hq[q];
      r.qid = q;
      r.k = C.queries[q].k;
      for (int sgn = 0; sgn < 2; ++sgn) {
        const uint64_t* p = h_qres + ((size_t)q * 2 + sgn) * 3;
        r.count[sgn] = p[0];
        r.hash_sum[sgn] = (flags & GAMMA_F_HASH) ? p[1] : 0;
        r.hash_xor[sgn] = (flags & GAMMA_F_HASH) ? p[2] : 0;
      }
      r.open_seeds = h_qres[(size_t)nq * 6 + q];
    }
    std::memset(out, 0, sizeof(*out));
    out->n_queries = nq;
    out->tuple_width = tw;
    out->queries = C.hq.data();
    out->n_tuples_found = (flags & GAMMA_F_TUPLES) ? h_ctr->tuples_found : 0;
    out->n_tuples = std::min<uint64_t>(out->n_tuples_found, tcap);
    out->tuples = (flags & GAMMA_F_TUPLES) ? (uint32_t*)C.tuples.p : nullptr;
    out->meta = (flags & GAMMA_F_TUPLES) ? (uint32_t*)C.tmeta.p : nullptr;
    out->ord = ((flags & GAMMA_F_TUPLES) && (flags & GAMMA_F_SEED_ATTR)) ? (uint32_t*)C.tord.p : nullptr;
    out->n_canonical = n_canon;
    if (flags & GAMMA_F_CANONICAL) {
      C.h_canon_lo.assign(h_clo ? h_clo : nullptr, h_clo ? h_clo + n_canon : nullptr);
      C.h_canon_hi.assign(h_clo ? h_clo + n_canon : nullptr, h_clo ? h_clo + 2 * (size_t)n_canon : nullptr);
      const uint8_t* sg = h_clo ? (const uint8_t*)(h_clo + 2 * (size_t)n_canon) : nullptr;
      C.h_canon_sign.assign(sg, sg ? sg + n_canon : nullptr);
      out->canon_lo = C.h_canon_lo.data();
      out->canon_hi = C.h_canon_hi.data();
      out->canon_sign = C.h_canon_sign.data();
    }
    if (flags & GAMMA_F_PER_UPDATE) {
      C.h_upd_cnt.resize(n_canon);
      C.h_upd_sum.resize(n_canon);
      C.h_upd_xor.resize(n_canon);
      for (uint32_t i = 0; i < n_canon; ++i) {
        C.h_upd_cnt[i] = h_upd[3 * (size_t)i];
        C.h_upd_sum[i] = h_upd[3 * (size_t)i + 1];
        C.h_upd_xor[i] = h_upd[3 * (size_t)i + 2];
      }
      out->upd_count = C.h_upd_cnt.data();
      out->upd_hash_sum = C.h_upd_sum.data();
      out->upd_hash_xor = C.h_upd_xor.data();
      C.h_upd_open.assign(h_uopen, h_uopen ? h_uopen + n_canon : nullptr);
      out->upd_open = C.h_upd_open.data();
    }
    gamma_batch_stats& st = out->stats;
    st.n_input = n_upd;
    st.n_canonical = n_canon;
    st.n_insert = n_insert;
    st.n_delete = n_delete;
    st.n_noop = hc.n_noop;
    st.n_duplicate = hc.n_dup;
    st.n_touched = n_touched;
    st.n_groups = n_groups;
    st.n_seeds = h_ctr->n_seeds;
    st.dfs_nodes = h_ctr->dfs_nodes;
    st.steals = h_ctr->steals;
    st.cand_scanned = h_ctr->cand_scanned;
    st.cyc_idle = h_ctr->cyc[0];
    st.cyc_init = h_ctr->cyc[1];
    st.cyc_inner = h_ctr->cyc[2];
    st.cyc_leaf = h_ctr->cyc[3];
    st.cyc_handover = h_ctr->cyc[4];
    st.tasks_received = h_ctr->cyc[5];
    st.seeds_started = std::min<uint64_t>(h_ctr->seed_head, h_ctr->n_seeds);
    st.bytes_alg_dfs = (h_ctr->bytes_alg + 4) / 8;  // the kernel counts eighths of a byte
    // merge: read old rows, write R1 and R2; commit: row pointers only
    st.bytes_alg_update = (r1_total - 2ull * n_insert) * 4 + r1_total * 4 + r2_total * 4 + (uint64_t)n_upd * 9;
    float ms = 0;
    auto el = [&](int a, int b) {
      float t = 0;
      (void)hipEventElapsedTime(&t, C.ev[a], C.ev[b]);
      return t;
    };
    st.ms_canon = el(0, 1);
    st.ms_merge = el(1, 2);
    st.ms_filter = el(2, 3);
    st.ms_seed = el(3, 4);
    st.ms_dfs = el(4, 5);
    st.ms_commit = el(5, 6);
    ms = el(0, 7);
    st.ms_total = ms;
    if (h_ctr->aborted || h_ctr->timed_out) {
      // rows were put back on the device: the graph is as before the batch
      C.has_result = false;
      return fail(c, GAMMA_ETIMEDOUT, "apply_batch: search deadline exceeded; batch not committed");
    }
    if (!dry) C.live = C.live + 2ull * n_insert - 2ull * n_delete;
    C.has_result = true;
    C.last_tuples = out->n_tuples;
    C.last_twidth = tw;
    C.last_has_ord = out->ord != nullptr;
    return out->n_tuples < out->n_tuples_found ? GAMMA_TRUNCATED : GAMMA_OK;
  });
}

}  // extern "C"

namespace gm {
uint64_t ctx_tuple_capacity(const gamma_ctx* c) { return c ? c->opt.tuple_capacity : 0; }

bool ctx_has_graph(const gamma_ctx* c, uint32_t* n, uint32_t* n_el) {
  if (!c || !c->has_graph) return false;
  if (n) *n = c->n;
  if (n_el) *n_el = c->n_el;
  return true;
}
}  // namespace gm

extern "C" {

gamma_status gamma_apply_batch(gamma_ctx* c, uint32_t n_upd, const uint32_t* src, const uint32_t* dst,
                               const uint8_t* op, gamma_mem where, uint32_t flags, gamma_batch_result* out) {
  return gamma_apply_batch_el(c, n_upd, src, dst, op, nullptr, where, flags, out);
}

gamma_status gamma_apply_batch_noalloc(gamma_ctx* c, uint32_t n_upd, const uint32_t* src, const uint32_t* dst,
                                       const uint8_t* op, gamma_mem where, uint32_t flags,
                                       gamma_batch_result* out) {
  if (!c) return GAMMA_EINVAL;
  if (flags & (GAMMA_F_TUPLES | GAMMA_F_SEED_ATTR))
    return fail(c, GAMMA_EUNSUPPORTED, "apply_batch_noalloc: counts, checksums and attribution only (no TUPLES)");
  void* base = scratch_of(c->device);
  if (!base) {
    c->last_error = std::string("apply_batch_noalloc: no scratch address on this device: ") +
                    hipGetErrorString(g_scratch_err[c->device >= 0 && c->device < NOALLOC_MAX_DEVICES ? c->device : 0]);
    return GAMMA_EDEVICE;
  }
  NoAllocArena na;
  na.base = (char*)base;
  na.cap = NOALLOC_SCRATCH_BYTES;
  na.given.reserve(64);
  c->na = &na;
  const gamma_status st = gamma_apply_batch_el(c, n_upd, src, dst, op, nullptr, where, flags, out);
  c->na = nullptr;
  return st;
}

gamma_status gamma_apply_batch_vertices(gamma_ctx* c, uint32_t n_upd, const uint32_t* src, const uint32_t* dst,
                                        const uint8_t* op, const uint32_t* elab, uint32_t n_vdel,
                                        const uint32_t* vdel, gamma_mem where, uint32_t flags,
                                        gamma_batch_result* out) {
  size_t N = 0;  // explicit updates + expanded vertex deletions
  const gamma_status st = guarded(c, [&]() -> gamma_status {
    if (!out) return fail(c, GAMMA_EINVAL, "apply_batch_vertices: null result");
    if (!c->has_graph) return fail(c, GAMMA_ESTATE, "apply_batch_vertices: no graph loaded");
    if (n_upd > (1u << 20) || n_vdel > (1u << 20)) return fail(c, GAMMA_EINVAL, "apply_batch_vertices: too many updates");
    if ((n_upd && (!src || !dst || !op)) || (n_vdel && !vdel))
      return fail(c, GAMMA_EINVAL, "apply_batch_vertices: null arrays");
    chk(hipSetDevice(c->device), "set device");
    gamma_ctx& C = *c;
    hipStream_t s = C.stream;
    const uint32_t* d_vdel = stage_in<uint32_t>(c, C.vx_del, vdel, n_vdel, where);
    uint64_t* len = C.ensure<uint64_t>(C.vx_len, std::max<uint32_t>(n_vdel, 1));
    uint64_t* offs = C.ensure<uint64_t>(C.vx_off, (size_t)n_vdel + 1);
    // word 0: error flags; words 1..: the deleted-vertex bit map
    const size_t mwords = ((size_t)C.n + 31) / 32;
    uint32_t* err = C.ensure<uint32_t>(C.vx_mark, 1 + mwords);
    uint32_t* mark = err + 1;
    gm::fill_u32(err, 0, 1 + mwords, s);
    gm::launch_vdel_len(C.G(), d_vdel, n_vdel, len, mark, err, s);
    const uint32_t* e_src = stage_in<uint32_t>(c, C.vx_src, src, n_upd, where);
    const uint32_t* e_dst = stage_in<uint32_t>(c, C.vx_dst, dst, n_upd, where);
    const uint8_t* e_op = stage_in<uint8_t>(c, C.vx_op, op, n_upd, where);
    gm::launch_vdel_check(e_src, e_dst, e_op, n_upd, C.n, mark, err, s);
    C.scan64(len, offs, n_vdel);
    uint64_t total = 0;
    uint32_t herr = 0;
    if (n_vdel) chk(hipMemcpyAsync(&total, offs + n_vdel, 8, hipMemcpyDeviceToHost, s), "d2h");
    chk(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s), "d2h");
    chk(hipStreamSynchronize(s), "sync");
    if (herr & GM_ERR_RANGE) return fail(c, GAMMA_EINVAL, "apply_batch_vertices: vertex id out of range");
    if (herr & GM_ERR_CONFLICT)
      return fail(c, GAMMA_ECONFLICT, "apply_batch_vertices: an insertion touches a deleted vertex");
    if ((uint64_t)n_upd + total > (1u << 20))
      return fail(c, GAMMA_EINVAL, "apply_batch_vertices: more than 2^20 updates after expanding vertex deletions");
    N = (size_t)n_upd + total;
    uint32_t* xs = C.ensure<uint32_t>(C.vx_src, std::max<size_t>(N, 1));
    uint32_t* xd = C.ensure<uint32_t>(C.vx_dst, std::max<size_t>(N, 1));
    uint8_t* xo = C.ensure<uint8_t>(C.vx_op, std::max<size_t>(N, 1));
    // with edge labels the merged batch carries them: the explicit ones (0
    // if none were given), then each expanded edge's own
    uint32_t* xe = C.elb ? C.ensure<uint32_t>(C.vx_el, std::max<size_t>(N, 1)) : nullptr;
    const hipMemcpyKind kind = where == GAMMA_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (n_upd) {
      chk(hipMemcpyAsync(xs, src, (size_t)n_upd * 4, kind, s), "copy");
      chk(hipMemcpyAsync(xd, dst, (size_t)n_upd * 4, kind, s), "copy");
      chk(hipMemcpyAsync(xo, op, n_upd, kind, s), "copy");
      if (xe && elab)
        chk(hipMemcpyAsync(xe, elab, (size_t)n_upd * 4, kind, s), "copy");
      else if (xe)
        gm::fill_u32(xe, 0, n_upd, s);
    }
    gm::launch_vdel_expand(C.G(), d_vdel, n_vdel, offs, xs + n_upd, xd + n_upd, xo + n_upd,
                           xe ? xe + n_upd : nullptr, s);
    chk(hipGetLastError(), "vertex deletion launch");
    return GAMMA_OK;
  });
  if (st != GAMMA_OK) return st;
  // the merged batch is device-resident and ordered on the context stream
  // after the expansion
  return gamma_apply_batch_el(c, (uint32_t)N, (const uint32_t*)c->vx_src.p, (const uint32_t*)c->vx_dst.p,
                              (const uint8_t*)c->vx_op.p, c->elb ? (const uint32_t*)c->vx_el.p : nullptr,
                              GAMMA_MEM_DEVICE, flags, out);
}

gamma_status gamma_add_vertices(gamma_ctx* c, uint32_t count, const uint32_t* labels, uint32_t* first_id) {
  return guarded(c, [&]() -> gamma_status {
    if (!c->has_graph) return fail(c, GAMMA_ESTATE, "add_vertices: no graph loaded");
    if (count == 0 || !labels) return fail(c, GAMMA_EINVAL, "add_vertices: nothing to add");
    const uint32_t n = c->n;
    if ((uint64_t)n + count >= 0x80000000ull) return fail(c, GAMMA_EINVAL, "add_vertices: n would reach 2^31");
    for (uint32_t i = 0; i < count; ++i)
      if (labels[i] > 0xFFFFu) return fail(c, GAMMA_EINVAL, "add_vertices: label >= 65536");
    // the new vertices are isolated: rebuild with the extended vertex set
    // (label-grouped internal ids interleave them with the old ones)
    const uint64_t nnz = c->live;
    std::vector<uint64_t> rp((size_t)n + count + 1);
    std::vector<uint32_t> col(std::max<uint64_t>(nnz, 1)), lab((size_t)n + count);
    std::vector<uint32_t> el(c->elb ? std::max<uint64_t>(nnz, 1) : 0);
    const uint32_t n_el = c->n_el;
    gamma_status st = gamma_export_graph_el(c, nullptr, nullptr, nullptr, rp.data(), col.data(), lab.data(),
                                            el.empty() ? nullptr : el.data());
    if (st < 0) return st;
    for (uint32_t i = 0; i < count; ++i) {
      rp[(size_t)n + 1 + i] = nnz;
      lab[(size_t)n + i] = labels[i];
    }
    st = load_graph_impl(c, n + count, nnz, rp.data(), nnz ? col.data() : nullptr, lab.data(),
                         el.empty() ? nullptr : el.data(), n_el, GAMMA_MEM_HOST);
    if (st < 0) return st;
    if (first_id) *first_id = n;
    return GAMMA_OK;
  });
}

gamma_status gamma_get_tuning(const gamma_ctx* c, gamma_tuning* out) {
  if (!c || !out) return GAMMA_EINVAL;
  *out = c->tun;
  return GAMMA_OK;
}

namespace {
bool tuning_ok(const gamma_tuning& t) {
  return t.waves_per_cu >= 1 && t.waves_per_cu <= 32 && (t.steal == 1 || t.steal == 2) &&
         t.poll_cycles >= 500 && t.poll_cycles <= 1000000 && t.split_inner >= 2 &&
         t.split_inner <= (1u << 20) && t.split_leaf >= 2 && t.split_leaf <= (1u << 20) &&
         (t.query_launch == 1 || t.query_launch == 2) && t.handover_gate >= 1 && t.handover_gate <= 1024 &&
         t.coalesced_search >= 1 && t.coalesced_search <= 3 && t.group_seeds >= 1 && t.group_seeds <= 3 &&
         t.shared_leaf >= 1 && t.shared_leaf <= 3;
}
}  // namespace

gamma_status gamma_set_tuning(gamma_ctx* c, const gamma_tuning* in) {
  if (!c || !in) return GAMMA_EINVAL;
  gamma_tuning t = c->tun;
  if (in->waves_per_cu) t.waves_per_cu = in->waves_per_cu;
  if (in->steal) t.steal = in->steal;
  if (in->poll_cycles) t.poll_cycles = in->poll_cycles;
  if (in->split_inner) t.split_inner = in->split_inner;
  if (in->split_leaf) t.split_leaf = in->split_leaf;
  if (in->query_launch) t.query_launch = in->query_launch;
  if (in->handover_gate) t.handover_gate = in->handover_gate;
  if (in->coalesced_search) t.coalesced_search = in->coalesced_search;
  if (in->group_seeds) t.group_seeds = in->group_seeds;
  if (in->shared_leaf) t.shared_leaf = in->shared_leaf;
  if (!tuning_ok(t)) return fail(c, GAMMA_EINVAL, "set_tuning: value out of range");
  c->tun = t;
  return GAMMA_OK;
}

gamma_status gamma_set_query_active(gamma_ctx* c, uint32_t qid, uint32_t active) {
  if (!c) return GAMMA_EINVAL;
  return guarded(c, [&]() -> gamma_status {
    if (qid >= c->queries.size()) return fail(c, GAMMA_EINVAL, "set_query_active: no such query");
    const bool paused = active == 0;
    if (c->queries[qid].paused == paused) return GAMMA_OK;
    chk(hipSetDevice(c->device), "set device");
    c->queries[qid].paused = paused;
    try {
      c->upload_plans();
    } catch (const StatusError&) {
      c->queries[qid].paused = !paused;
      throw;
    }
    return GAMMA_OK;
  });
}

gamma_status gamma_set_deadline(gamma_ctx* c, uint32_t deadline_ms) {
  if (!c) return GAMMA_EINVAL;
  c->opt.deadline_ms = deadline_ms;
  return GAMMA_OK;
}

gamma_status gamma_autotune(gamma_ctx* c, uint32_t n_upd, const uint32_t* src, const uint32_t* dst,
                            const uint8_t* op, gamma_mem where, uint32_t flags, uint32_t max_points,
                            uint32_t reps, gamma_tuning* best, double* best_ms, double* base_ms) {
  if (!c || !best) return GAMMA_EINVAL;
  if (max_points < 1 || max_points > 64 || reps < 1 || reps > 9)
    return fail(c, GAMMA_EINVAL, "autotune: max_points must be 1..64 and reps 1..9");
  flags = (flags | GAMMA_F_DRY_RUN) & ~(uint32_t)GAMMA_F_TUPLES;
  std::vector<std::pair<gamma_tuning, double>> seen;
  auto same = [](const gamma_tuning& a, const gamma_tuning& b) {
    return a.waves_per_cu == b.waves_per_cu && a.steal == b.steal && a.poll_cycles == b.poll_cycles &&
           a.split_inner == b.split_inner && a.split_leaf == b.split_leaf && a.query_launch == b.query_launch &&
           a.handover_gate == b.handover_gate && a.coalesced_search == b.coalesced_search &&
           a.group_seeds == b.group_seeds && a.shared_leaf == b.shared_leaf;
  };
  gamma_status err = GAMMA_OK;
  // median device time of `reps` dry runs at tuning t (< 0: failed)
  auto eval = [&](const gamma_tuning& t) -> double {
    for (auto& p : seen)
      if (same(p.first, t)) return p.second;
    if ((uint32_t)seen.size() >= max_points || err != GAMMA_OK) return -1.0;
    c->tun = t;
    std::vector<double> ms;
    for (uint32_t r = 0; r < reps; ++r) {
      gamma_batch_result res;
      const gamma_status st = gamma_apply_batch(c, n_upd, src, dst, op, where, flags, &res);
      if (st < 0) {
        err = st;
        return -1.0;
      }
      ms.push_back(res.stats.ms_total);
    }
    std::sort(ms.begin(), ms.end());
    const double m = ms[ms.size() / 2];
    seen.push_back({t, m});
    return m;
  };
  const gamma_tuning start = c->tun;
  gamma_tuning cur = start;
  double cur_ms = eval(cur);
  if (cur_ms < 0) {
    c->tun = start;
    return err != GAMMA_OK ? err : GAMMA_EINVAL;
  }
  if (base_ms) *base_ms = cur_ms;
  const uint32_t wpc_v[] = {4, 8, 12, 16, 24};
  const uint32_t poll_v[] = {1500, 3000, 6000, 12000, 24000};
  const uint32_t leaf_v[] = {128, 256, 512, 1024, 2048};
  const uint32_t inner_v[] = {64, 128, 256, 512};
  const uint32_t gate_v[] = {1, 2, 4, 8, 16};
  const bool many_q = c->queries.size() > 1;
  for (int pass = 0; pass < 3; ++pass) {
    bool moved = false;
    // one dimension at a time: keep a value only if it is at least 1% faster
    auto sweep = [&](uint32_t gamma_tuning::*f, const uint32_t* vals, int nv) {
      for (int i = 0; i < nv; ++i) {
        if (cur.*f == vals[i]) continue;
        gamma_tuning t = cur;
        t.*f = vals[i];
        const double m = eval(t);
        if (m >= 0 && m < 0.99 * cur_ms) {
          cur = t;
          cur_ms = m;
          moved = true;
        }
      }
    };
    const uint32_t ql_v[] = {1, 2}, steal_v[] = {1, 2}, cs_v[] = {2, 1, 3}, gs_v[] = {1, 2, 3};
    if (many_q) sweep(&gamma_tuning::query_launch, ql_v, 2);
    sweep(&gamma_tuning::coalesced_search, cs_v, 3);
    if (cur.query_launch == 1) sweep(&gamma_tuning::group_seeds, gs_v, 3);
    sweep(&gamma_tuning::steal, steal_v, 2);
    sweep(&gamma_tuning::waves_per_cu, wpc_v, 5);
    if (cur.steal == 1) {
      sweep(&gamma_tuning::handover_gate, gate_v, 5);
      sweep(&gamma_tuning::poll_cycles, poll_v, 5);
      sweep(&gamma_tuning::split_leaf, leaf_v, 5);
      sweep(&gamma_tuning::split_inner, inner_v, 4);
    }
    if (!moved || err != GAMMA_OK || (uint32_t)seen.size() >= max_points) break;
  }
  if (err != GAMMA_OK && err != GAMMA_ETIMEDOUT) {
    c->tun = start;
    return err;
  }
  c->tun = cur;
  *best = cur;
  if (best_ms) *best_ms = cur_ms;
  return GAMMA_OK;
}

gamma_status gamma_copy_tuples(gamma_ctx* c, uint32_t* tuples, uint32_t* meta, uint32_t* ord,
                               uint64_t max_records, gamma_mem where) {
  return guarded(c, [&]() -> gamma_status {
    if (!c->has_result) return fail(c, GAMMA_ESTATE, "copy_tuples: no batch result");
    uint64_t nrec = std::min<uint64_t>(max_records, c->last_tuples);
    hipMemcpyKind kind = where == GAMMA_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (nrec && tuples)
      chk(hipMemcpyAsync(tuples, c->tuples.p, nrec * c->last_twidth * 4, kind, c->stream), "copy");
    if (nrec && meta) chk(hipMemcpyAsync(meta, c->tmeta.p, nrec * 4, kind, c->stream), "copy");
    if (nrec && ord) {
      if (!c->last_has_ord) return fail(c, GAMMA_ESTATE, "copy_tuples: no seed attribution stored");
      chk(hipMemcpyAsync(ord, c->tord.p, nrec * 4, kind, c->stream), "copy");
    }
    chk(hipStreamSynchronize(c->stream), "sync");
    return GAMMA_OK;
  });
}

gamma_status gamma_result_release(gamma_ctx* c, gamma_batch_result* res) {
  return guarded(c, [&]() -> gamma_status {
    c->has_result = false;
    if (res) std::memset(res, 0, sizeof(*res));
    return GAMMA_OK;
  });
}

gamma_status gamma_export_graph_el(gamma_ctx* c, uint32_t* n_out, uint64_t* nnz_out, uint32_t* n_elabels_out,
                                   uint64_t* row_ptr, uint32_t* col, uint32_t* labels, uint32_t* elabels) {
  return guarded(c, [&]() -> gamma_status {
    if (!c->has_graph) return fail(c, GAMMA_ESTATE, "export_graph: no graph loaded");
    if (n_out) *n_out = c->n;
    if (nnz_out) *nnz_out = c->live;
    if (n_elabels_out) *n_elabels_out = c->n_el;
    if (!col && !row_ptr && !labels && !elabels) return GAMMA_OK;
    gamma_ctx& C = *c;
    hipStream_t s = C.stream;
    const uint32_t n = C.n;
    const int ib = C.idbits;
    const uint64_t nnz = C.live;
    const uint32_t elb = C.elb, rows = C.rows();
    uint64_t* deg = C.ensure<uint64_t>(C.tmp64a, (size_t)n + 1);
    if (elb)
      gm::launch_deg_rows((const uint32_t*)C.row_len.p, (const uint32_t*)C.old_of_new.p, n, elb, deg, s);
    else
      gm::launch_deg_mapped(nullptr, (const uint32_t*)C.row_len.p, (const uint32_t*)C.old_of_new.p, n, deg, s);
    uint64_t* offs = C.ensure<uint64_t>(C.sizes, (size_t)n + 1);
    C.scan64(deg, offs, n);
    if (row_ptr) {
      chk(hipMemcpyAsync(row_ptr, offs, ((size_t)n + 1) * 8, hipMemcpyDeviceToHost, s), "d2h");
    }
    if (elb && (col || elabels) && nnz) {
      // rows (v, e) packed densely, keyed (old v, old w, e), sorted, split
      uint64_t* ek = C.ensure<uint64_t>(C.keys, nnz);
      uint64_t* et = C.ensure<uint64_t>(C.keys_tmp, nnz);
      uint64_t* ideg = C.ensure<uint64_t>(C.runvals, (size_t)rows + 1);
      gm::launch_deg_mapped(nullptr, (const uint32_t*)C.row_len.p, nullptr, rows, ideg, s);
      uint64_t* ioffs = C.ensure<uint64_t>(C.runscan, (size_t)rows + 1);
      C.scan64(ideg, ioffs, rows);
      gm::launch_row_keys_el((const uint64_t*)C.row_off.p, (const uint32_t*)C.row_len.p, (const uint32_t*)C.arena.p,
                             (const uint32_t*)C.old_of_new.p, rows, elb, ib, ioffs, ek, s);
      C.sort_keys(ek, et, nnz, 2 * ib + (int)elb);
      uint32_t* oc = C.ensure<uint32_t>(C.tmp32a, 2 * nnz);
      gm::launch_keys_split_el(ek, nnz, ib, elb, oc, oc + nnz, s);
      if (col) chk(hipMemcpyAsync(col, oc, nnz * 4, hipMemcpyDeviceToHost, s), "d2h");
      if (elabels) chk(hipMemcpyAsync(elabels, oc + nnz, nnz * 4, hipMemcpyDeviceToHost, s), "d2h");
    } else if (elabels && nnz) {
      std::fill(elabels, elabels + nnz, 0u);
    }
    if (!elb && col && nnz) {
      uint64_t* ek = C.ensure<uint64_t>(C.keys, nnz);
      uint64_t* et = C.ensure<uint64_t>(C.keys_tmp, nnz);
      // internal row offsets packed densely: scan of row_len in internal order
      uint64_t* ideg = C.ensure<uint64_t>(C.runvals, (size_t)n + 1);
      gm::launch_deg_mapped(nullptr, (const uint32_t*)C.row_len.p, nullptr, n, ideg, s);
      uint64_t* ioffs = C.ensure<uint64_t>(C.runscan, (size_t)n + 1);
      C.scan64(ideg, ioffs, n);
      gm::launch_csr_keys((const uint64_t*)C.row_off.p, (const uint32_t*)C.row_len.p, nullptr,
                          (const uint32_t*)C.arena.p, (const uint32_t*)C.old_of_new.p, n, ib, ioffs, ek, s);
      C.sort_keys(ek, et, nnz, 2 * ib);
      uint32_t* oc = C.ensure<uint32_t>(C.tmp32a, nnz);
      gm::launch_csr_extract(ek, nnz, (1ull << ib) - 1, oc, s);
      chk(hipMemcpyAsync(col, oc, nnz * 4, hipMemcpyDeviceToHost, s), "d2h");
    }
    chk(hipStreamSynchronize(s), "sync");
    if (labels) {
      std::vector<uint16_t> vl(n);
      std::vector<uint32_t> o2n(n);
      chk(hipMemcpy(vl.data(), C.vlabel.p, (size_t)n * 2, hipMemcpyDeviceToHost), "d2h");
      chk(hipMemcpy(o2n.data(), C.old_of_new.p, (size_t)n * 4, hipMemcpyDeviceToHost), "d2h");
      for (uint32_t v = 0; v < n; ++v) labels[o2n[v]] = vl[v];
    }
    chk(hipGetLastError(), "export launch");
    return GAMMA_OK;
  });
}

gamma_status gamma_export_graph(gamma_ctx* c, uint32_t* n_out, uint64_t* nnz_out, uint64_t* row_ptr,
                                uint32_t* col, uint32_t* labels) {
  return gamma_export_graph_el(c, n_out, nnz_out, nullptr, row_ptr, col, labels, nullptr);
}

// ------------------------------------------------------------------ host validators

gamma_status gamma_validate_graph(uint32_t n, uint64_t nnz, const uint64_t* rp, const uint32_t* col,
                                  const uint32_t* labels) {
  if (n == 0 || n >= 0x80000000u || !rp || !labels || (nnz && !col)) return GAMMA_EINVAL;
  if (rp[0] != 0 || rp[n] != nnz) return GAMMA_EINVAL;
  for (uint32_t v = 0; v < n; ++v) {
    if (labels[v] > 0xFFFFu) return GAMMA_EINVAL;
    if (rp[v] > rp[v + 1] || rp[v + 1] > nnz) return GAMMA_EINVAL;
  }
  for (uint32_t v = 0; v < n; ++v) {
    for (uint64_t j = rp[v]; j < rp[v + 1]; ++j) {
      uint32_t x = col[j];
      if (x >= n || x == v) return GAMMA_EINVAL;
      if (j > rp[v] && col[j - 1] >= x) return GAMMA_EINVAL;
      if (!std::binary_search(col + rp[x], col + rp[x + 1], v)) return GAMMA_EINVAL;
    }
  }
  return GAMMA_OK;
}

gamma_status gamma_validate_graph_el(uint32_t n, uint64_t nnz, const uint64_t* rp, const uint32_t* col,
                                     const uint32_t* labels, const uint32_t* elabels, uint32_t n_elabels) {
  if (n_elabels == 0 || n_elabels > GAMMA_MAX_EDGE_LABELS || (!elabels && n_elabels != 1)) return GAMMA_EINVAL;
  const gamma_status st = gamma_validate_graph(n, nnz, rp, col, labels);
  if (st != GAMMA_OK || !elabels) return st;
  // every label in range and equal on the mirror entry (the graph is simple)
  for (uint32_t v = 0; v < n; ++v)
    for (uint64_t j = rp[v]; j < rp[v + 1]; ++j) {
      if (elabels[j] >= n_elabels) return GAMMA_EINVAL;
      const uint32_t x = col[j];
      const uint32_t* p = std::lower_bound(col + rp[x], col + rp[x + 1], v);
      if (elabels[p - col] != elabels[j]) return GAMMA_EINVAL;
    }
  return GAMMA_OK;
}

gamma_status gamma_validate_batch_el(uint32_t n, uint32_t n_elabels, uint32_t n_upd, const uint32_t* src,
                                     const uint32_t* dst, const uint8_t* op, const uint32_t* elab) {
  if (n_elabels == 0 || n_elabels > GAMMA_MAX_EDGE_LABELS) return GAMMA_EINVAL;
  const gamma_status st = gamma_validate_batch(n, n_upd, src, dst, op);
  if (st != GAMMA_OK || !elab) return st;
  std::vector<std::pair<uint64_t, uint32_t>> keys;  // pair, label << 1 | op
  keys.reserve(n_upd);
  for (uint32_t i = 0; i < n_upd; ++i) {
    if (elab[i] >= n_elabels) return GAMMA_EINVAL;
    const uint64_t lo = std::min(src[i], dst[i]), hi = std::max(src[i], dst[i]);
    keys.push_back({(lo << 32) | hi, (elab[i] << 1) | (op[i] ? 1u : 0u)});
  }
  std::sort(keys.begin(), keys.end());
  for (size_t i = 1; i < keys.size(); ++i)
    if (keys[i].first == keys[i - 1].first && keys[i].second != keys[i - 1].second) return GAMMA_ECONFLICT;
  return GAMMA_OK;
}

gamma_status gamma_validate_query(uint32_t k, const uint32_t* qlabels, uint32_t m, const uint32_t* qedges) {
  return (gamma_status)gm::validate_query(k, qlabels, m, qedges, nullptr);
}

gamma_status gamma_describe_query(uint32_t k, const uint32_t* qlabels, uint32_t m, const uint32_t* qedges,
                                  const uint32_t* qelabels, uint32_t max_plans, gamma_plan_info* plans,
                                  uint32_t* n_plans, uint32_t max_perms, uint32_t* perms, uint32_t* n_perms) {
  const int st = gm::validate_query(k, qlabels, m, qedges, nullptr);
  if (st != GAMMA_OK) return (gamma_status)st;
  for (uint32_t e = 0; qelabels && e < m; ++e)
    if (qelabels[e] >= GAMMA_MAX_EDGE_LABELS) return GAMMA_EINVAL;
  if (!n_plans || !n_perms) return GAMMA_EINVAL;
  gm::HostQuery q;
  q.k = k;
  q.labels.assign(qlabels, qlabels + k);
  for (uint32_t e = 0; e < m; ++e) q.edges.push_back({qedges[2 * e], qedges[2 * e + 1]});
  q.elabels.assign(m, 0);
  if (qelabels) q.elabels.assign(qelabels, qelabels + m);
  gm::plan_query(q, 0, std::vector<uint64_t>());
  const uint32_t np = (uint32_t)q.plans.size();
  const uint32_t n0 = (uint32_t)q.perms.size(), nt = n0 + (uint32_t)q.cperms.size();
  *n_plans = np;
  *n_perms = nt;
  if (np > max_plans || nt > max_perms || (np && !plans) || (nt && !perms)) return GAMMA_EINVAL;
  for (uint32_t i = 0; i < np; ++i) {
    const GmPlan& p = q.plans[i];
    gamma_plan_info& o = plans[i];
    std::memset(&o, 0, sizeof(o));
    o.x = p.x;
    o.y = p.y;
    o.n_perm = p.n_perm;
    o.perm_first = p.perm_base;
    o.n_core = p.n_core;
    o.n_cperm = p.n_cperm;
    o.cperm_first = n0 + p.cperm_base;
    for (uint32_t l = 0; l < GM_MAX_K; ++l) {
      o.order[l] = l < k ? p.order[l] : 0u;
      o.omask[l] = p.omask[l];
    }
  }
  for (uint32_t j = 0; j < nt; ++j) {
    const GmPerm& g = j < n0 ? q.perms[j] : q.cperms[j - n0];
    for (uint32_t v = 0; v < GM_MAX_K; ++v) perms[GM_MAX_K * j + v] = g.fwd[v];
  }
  return GAMMA_OK;
}

gamma_status gamma_validate_batch(uint32_t n, uint32_t n_upd, const uint32_t* src, const uint32_t* dst,
                                  const uint8_t* op) {
  if (n_upd > (1u << 20)) return GAMMA_EINVAL;
  if (n_upd && (!src || !dst || !op)) return GAMMA_EINVAL;
  std::vector<uint64_t> keys;
  keys.reserve(n_upd);
  for (uint32_t i = 0; i < n_upd; ++i) {
    if (src[i] >= n || dst[i] >= n || src[i] == dst[i]) return GAMMA_EINVAL;
    uint64_t lo = std::min(src[i], dst[i]), hi = std::max(src[i], dst[i]);
    keys.push_back((lo << 33) | (hi << 1) | (op[i] ? 1u : 0u));
  }
  std::sort(keys.begin(), keys.end());
  for (size_t i = 1; i < keys.size(); ++i)
    if ((keys[i] >> 1) == (keys[i - 1] >> 1) && keys[i] != keys[i - 1]) return GAMMA_ECONFLICT;
  return GAMMA_OK;
}

}  // extern "C"
