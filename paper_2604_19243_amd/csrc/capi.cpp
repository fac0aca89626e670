// The extern "C" boundary: status codes, thread-local messages and the handle
// registry.
//
// Handles are opaque identifiers (a serial number and a kind tag), not
// pointers, and serial numbers are never reused: a destroyed handle, or a value
// this library never returned, is found missing from the registry and the
// call fails with KIFMM_E_STATE instead of touching freed memory.  A call takes
// a reference on the object for its duration, so an object destroyed by
// another thread meanwhile stays alive until the call returns.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>

#include "common.hpp"
#include "plan.hpp"

namespace kifmm {
namespace {
thread_local std::string g_last_error;
}
void set_last_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }
}  // namespace kifmm

using namespace kifmm;

namespace {

template <class F>
kifmm_status guarded(F&& body) {
  try {
    set_last_error("");
    body();
    return KIFMM_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.status;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return KIFMM_E_NOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return KIFMM_E_INVALID;
  } catch (...) {
    set_last_error("unknown error");
    return KIFMM_E_INVALID;
  }
}

enum Kind : uint64_t { kTree = 1, kOps = 2, kPlan = 3 };
const char* kind_name(Kind k) { return k == kTree ? "tree" : k == kOps ? "ops" : "plan"; }

// Live handles: value (serial << 4 | kind) -> object.  The registry holds the
// caller's reference of each object.
struct Registry {
  std::mutex mu;
  std::unordered_map<uint64_t, Object*> live;
  uint64_t next = 1;
};
Registry& registry() {
  static Registry r;
  return r;
}

void* add_handle(Kind k, Object* obj) {
  Registry& r = registry();
  std::lock_guard<std::mutex> lock(r.mu);
  const uint64_t h = (r.next++ << 4) | (uint64_t)k;
  r.live.emplace(h, obj);
  return reinterpret_cast<void*>((uintptr_t)h);
}

// A reference on a live object of kind K for the duration of one call.
template <class T>
struct Held {
  T* p = nullptr;
  Held(const Held&) = delete;
  Held& operator=(const Held&) = delete;
  explicit Held(T* q) : p(q) {}
  Held(Held&& o) noexcept : p(o.p) { o.p = nullptr; }
  ~Held() { release(p); }
  T* operator->() const { return p; }
  T& operator*() const { return *p; }
};

template <class T>
Held<T> hold(const void* handle, Kind k) {
  require(handle != nullptr, std::string("null ") + kind_name(k) + " handle");
  Registry& r = registry();
  std::lock_guard<std::mutex> lock(r.mu);
  const uint64_t h = (uint64_t)(uintptr_t)handle;
  auto it = r.live.find(h);
  if ((h & 15u) != (uint64_t)k || it == r.live.end())
    fail(KIFMM_E_STATE, std::string("the ") + kind_name(k) + " handle is destroyed or was not made by this library");
  it->second->refs.fetch_add(1);
  return Held<T>(static_cast<T*>(it->second));
}

void drop_handle(const void* handle, Kind k) {
  require(handle != nullptr, std::string("null ") + kind_name(k) + " handle");
  Object* obj = nullptr;
  {
    Registry& r = registry();
    std::lock_guard<std::mutex> lock(r.mu);
    const uint64_t h = (uint64_t)(uintptr_t)handle;
    auto it = r.live.find(h);
    if ((h & 15u) != (uint64_t)k || it == r.live.end())
      fail(KIFMM_E_STATE, std::string("the ") + kind_name(k) + " handle is already destroyed or was not made by this library");
    obj = it->second;
    r.live.erase(it);
  }
  release(obj);
}

void copy_out(const double* src, int64_t count, double* out, int64_t capacity) {
  require(out != nullptr, "output is null");
  require(capacity >= count, "capacity too small: need " + std::to_string(count));
  std::memcpy(out, src, count * sizeof(double));
}

std::atomic<int64_t> g_device_limit{0};

}  // namespace

namespace kifmm {
int64_t device_memory_limit() { return g_device_limit.load(); }
}  // namespace kifmm

extern "C" {

int kifmm_abi_version(void) { return KIFMM_ABI_VERSION; }

const char* kifmm_last_error(void) { return last_error_cstr(); }

kifmm_status kifmm_tree_build(const float* xyz, int64_t n, int depth, const double* cube, void* stream,
                              kifmm_tree* out) {
  return guarded([&] {
    require(out != nullptr, "out is null");
    *out = nullptr;
    Tree* t = build_tree_device(xyz, n, depth, cube, (hipStream_t)stream);
    *out = reinterpret_cast<kifmm_tree>(add_handle(kTree, t));
  });
}

kifmm_status kifmm_tree_build_host(const float* xyz, int64_t n, int depth, const double* cube, kifmm_tree* out) {
  return guarded([&] {
    require(out != nullptr, "out is null");
    *out = nullptr;
    Tree* t = build_tree(xyz, n, depth, cube);
    *out = reinterpret_cast<kifmm_tree>(add_handle(kTree, t));
  });
}

kifmm_status kifmm_tree_stats_get(kifmm_tree tree, kifmm_tree_stats* out) {
  return guarded([&] {
    Held<Tree> t = hold<Tree>(tree, kTree);
    require(out != nullptr, "out is null");
    std::memset(out, 0, sizeof(*out));
    out->n = t->n;
    out->depth = t->depth;
    out->max_leaf = t->max_leaf;
    out->nonempty_leaves = (int64_t)t->keys[t->depth].size();
    for (int l = 0; l <= t->depth; ++l) out->nonempty_boxes[l] = (int64_t)t->keys[l].size();
    for (int d = 0; d < 3; ++d) out->center[d] = t->center[d];
    out->half_width = t->half;
  });
}

kifmm_status kifmm_tree_get_order(kifmm_tree tree, int64_t* order) {
  return guarded([&] {
    Held<Tree> t = hold<Tree>(tree, kTree);
    require(order != nullptr, "order is null");
    std::copy(t->order.begin(), t->order.end(), order);
  });
}

kifmm_status kifmm_tree_get_leaf_coords(kifmm_tree tree, int32_t* ijk) {
  return guarded([&] {
    Held<Tree> t = hold<Tree>(tree, kTree);
    require(ijk != nullptr, "ijk is null");
    std::copy(t->ijk.begin(), t->ijk.end(), ijk);
  });
}

kifmm_status kifmm_tree_destroy(kifmm_tree tree) {
  return guarded([&] { drop_handle(tree, kTree); });
}

kifmm_status kifmm_ops_precompute(int p, double alpha_inner, double alpha_outer, double eps_pinv, double eps_svd,
                                  kifmm_ops* out) {
  return guarded([&] {
    require(out != nullptr, "out is null");
    *out = nullptr;
    Ops* o = precompute_ops(p, alpha_inner, alpha_outer, eps_pinv, eps_svd);
    *out = reinterpret_cast<kifmm_ops>(add_handle(kOps, o));
  });
}

kifmm_status kifmm_ops_get_info(kifmm_ops ops, kifmm_ops_info* out) {
  return guarded([&] {
    Held<Ops> o = hold<Ops>(ops, kOps);
    require(out != nullptr, "out is null");
    std::memset(out, 0, sizeof(*out));
    out->p = o->p;
    out->n_surface = o->n;
    out->rank_m2l = o->k;
    out->rank_c2e = o->kc;
    out->n_m2l_offsets = kNumOffsets;
    out->eps_pinv = o->eps_pinv;
    out->eps_svd = o->eps_svd;
    out->alpha_inner = o->alpha_inner;
    out->alpha_outer = o->alpha_outer;
  });
}

kifmm_status kifmm_ops_get_matrix(kifmm_ops ops, int which, int index, double* out, int64_t capacity) {
  return guarded([&] {
    Held<Ops> o = hold<Ops>(ops, kOps);
    const int64_t n = o->n, k = o->k;
    switch (which) {
      case KIFMM_OP_SURFACE: copy_out(o->surf.data(), 3 * n, out, capacity); break;
      case KIFMM_OP_UC2E: copy_out(o->uc2e.data(), n * n, out, capacity); break;
      case KIFMM_OP_DC2E: copy_out(o->dc2e.data(), n * n, out, capacity); break;
      case KIFMM_OP_M2M:
      case KIFMM_OP_L2L:
        require(index >= 0 && index < 8, "child position must be in [0, 8)");
        copy_out((which == KIFMM_OP_M2M ? o->m2m : o->l2l).data() + (size_t)index * n * n, n * n, out, capacity);
        break;
      case KIFMM_OP_M2L_U: copy_out(o->mu.data(), n * k, out, capacity); break;
      case KIFMM_OP_M2L_V: copy_out(o->mv.data(), n * k, out, capacity); break;
      case KIFMM_OP_M2L_CORE:
        require(index >= 0 && index < kNumOffsets, "offset index must be in [0, 316)");
        copy_out(o->cores.data() + (size_t)index * k * k, k * k, out, capacity);
        break;
      case KIFMM_OP_M2L_OFFSET: {
        require(index >= 0 && index < kNumOffsets, "offset index must be in [0, 316)");
        const double t[3] = {(double)o->offsets[3 * index], (double)o->offsets[3 * index + 1],
                             (double)o->offsets[3 * index + 2]};
        copy_out(t, 3, out, capacity);
        break;
      }
      case KIFMM_OP_M2L_POST: copy_out(o->post.data(), n * k, out, capacity); break;
      default: fail(KIFMM_E_INVALID, "unknown operator kind");
    }
  });
}

kifmm_status kifmm_ops_destroy(kifmm_ops ops) {
  return guarded([&] { drop_handle(ops, kOps); });
}

kifmm_status kifmm_plan_create(kifmm_tree tree, kifmm_ops ops, int nrhs, unsigned flags, void* stream,
                               kifmm_plan* out) {
  return guarded([&] {
    require(out != nullptr, "out is null");
    *out = nullptr;
    Held<Tree> t = hold<Tree>(tree, kTree);
    Held<Ops> o = hold<Ops>(ops, kOps);
    Plan* p = create_plan(t.p, o.p, nrhs, flags, (hipStream_t)stream);
    *out = reinterpret_cast<kifmm_plan>(add_handle(kPlan, p));
  });
}

kifmm_status kifmm_plan_workspace_bytes(kifmm_tree tree, kifmm_ops ops, int nrhs, unsigned flags, int64_t* bytes) {
  return guarded([&] {
    require(bytes != nullptr, "bytes is null");
    Held<Tree> t = hold<Tree>(tree, kTree);
    Held<Ops> o = hold<Ops>(ops, kOps);
    *bytes = plan_workspace_bytes(t.p, o.p, nrhs, flags);
  });
}

kifmm_status kifmm_set_device_memory_limit(int64_t bytes) {
  return guarded([&] {
    require(bytes >= 0, "the device memory limit must be >= 0 (0: no limit)");
    g_device_limit.store(bytes);
  });
}

kifmm_status kifmm_evaluate(kifmm_plan plan, const float* charges, float* potential, float* gradient, void* stream) {
  return guarded([&] {
    Held<Plan> p = hold<Plan>(plan, kPlan);
    evaluate_plan(p.p, charges, potential, gradient, (hipStream_t)stream);
  });
}

kifmm_status kifmm_evaluate_vjp(kifmm_plan plan, const float* charges, const float* weights, const float* field,
                                float* grad_charges, float* grad_points, void* stream) {
  return guarded([&] {
    Held<Plan> p = hold<Plan>(plan, kPlan);
    evaluate_vjp(p.p, charges, weights, field, grad_charges, grad_points, (hipStream_t)stream);
  });
}

kifmm_status kifmm_evaluate_vjp_noalloc(kifmm_plan plan, const float* charges, const float* weights,
                                        const float* field, float* grad_charges, float* grad_points, void* stream) {
  return guarded([&] {
    Held<Plan> p = hold<Plan>(plan, kPlan);
    evaluate_vjp_noalloc(p.p, charges, weights, field, grad_charges, grad_points, (hipStream_t)stream);
  });
}

kifmm_status kifmm_plan_destroy(kifmm_plan plan) {
  return guarded([&] { drop_handle(plan, kPlan); });
}

kifmm_status kifmm_plan_set_timing(kifmm_plan plan, int enable) {
  return guarded([&] {
    Held<Plan> p = hold<Plan>(plan, kPlan);
    p->set_timing(enable != 0);
  });
}

kifmm_status kifmm_plan_get_stage_times(kifmm_plan plan, double* ms, int64_t* counts, int reset) {
  return guarded([&] {
    Held<Plan> p = hold<Plan>(plan, kPlan);
    require(ms != nullptr && counts != nullptr, "output is null");
    p->collect_times();
    for (int s = 0; s < KIFMM_N_STAGES; ++s) {
      ms[s] = p->stage_ms[s];
      counts[s] = p->stage_count[s];
      if (reset) {
        p->stage_ms[s] = 0.0;
        p->stage_count[s] = 0;
      }
    }
  });
}

kifmm_status kifmm_plan_get_stats(kifmm_plan plan, int64_t* stats, int count) {
  return guarded([&] {
    Held<Plan> p = hold<Plan>(plan, kPlan);
    require(stats != nullptr && count >= 0, "stats is null or count is negative");
    int64_t v[KIFMM_N_STATS];
    plan_stats(p.p, v);
    for (int i = 0; i < count && i < KIFMM_N_STATS; ++i) stats[i] = v[i];
  });
}

kifmm_status kifmm_plan_read_density(kifmm_plan plan, int kind, int level, float* host_out, int64_t capacity) {
  return guarded([&] {
    Held<Plan> p = hold<Plan>(plan, kPlan);
    read_density(p.p, kind, level, host_out, capacity);
  });
}

}  // extern "C"
