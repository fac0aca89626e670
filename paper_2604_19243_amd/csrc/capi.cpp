// The extern "C" boundary: status codes, thread-local messages, handle checks.
#include <algorithm>
#include <cstring>
#include <new>
#include <string>

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

Tree* as_tree(kifmm_tree h) {
  require(h != nullptr, "null tree handle");
  return reinterpret_cast<Tree*>(h);
}
Ops* as_ops(kifmm_ops h) {
  require(h != nullptr, "null ops handle");
  return reinterpret_cast<Ops*>(h);
}
Plan* as_plan(kifmm_plan h) {
  require(h != nullptr, "null plan handle");
  return reinterpret_cast<Plan*>(h);
}

void copy_out(const double* src, int64_t count, double* out, int64_t capacity) {
  require(out != nullptr, "output is null");
  require(capacity >= count, "capacity too small: need " + std::to_string(count));
  std::memcpy(out, src, count * sizeof(double));
}

}  // namespace

extern "C" {

int kifmm_abi_version(void) { return KIFMM_ABI_VERSION; }

const char* kifmm_last_error(void) { return last_error_cstr(); }

kifmm_status kifmm_tree_build(const float* xyz, int64_t n, int depth, const double* cube, kifmm_tree* out) {
  return guarded([&] {
    require(out != nullptr, "out is null");
    *out = nullptr;
    *out = reinterpret_cast<kifmm_tree>(build_tree(xyz, n, depth, cube));
  });
}

kifmm_status kifmm_tree_get_info(kifmm_tree tree, kifmm_tree_info* out) {
  return guarded([&] {
    const Tree* t = as_tree(tree);
    require(out != nullptr, "out is null");
    std::memset(out, 0, sizeof(*out));
    out->n_points = t->n;
    out->depth = t->depth;
    out->max_leaf_points = t->max_leaf;
    out->nonempty_leaves = (int64_t)t->keys[t->depth].size();
    for (int l = 0; l <= t->depth; ++l) out->nonempty_boxes[l] = (int64_t)t->keys[l].size();
    for (int d = 0; d < 3; ++d) out->center[d] = t->center[d];
    out->half_width = t->half;
  });
}

kifmm_status kifmm_tree_get_order(kifmm_tree tree, int64_t* order) {
  return guarded([&] {
    const Tree* t = as_tree(tree);
    require(order != nullptr, "order is null");
    std::copy(t->order.begin(), t->order.end(), order);
  });
}

kifmm_status kifmm_tree_get_leaf_coords(kifmm_tree tree, int32_t* ijk) {
  return guarded([&] {
    const Tree* t = as_tree(tree);
    require(ijk != nullptr, "ijk is null");
    std::copy(t->ijk.begin(), t->ijk.end(), ijk);
  });
}

kifmm_status kifmm_tree_destroy(kifmm_tree tree) {
  return guarded([&] { release(as_tree(tree)); });
}

kifmm_status kifmm_ops_precompute(int p, double eps_pinv, double eps_svd, int rank, kifmm_ops* out) {
  return guarded([&] {
    require(out != nullptr, "out is null");
    *out = nullptr;
    *out = reinterpret_cast<kifmm_ops>(precompute_ops(p, eps_pinv, eps_svd, rank));
  });
}

kifmm_status kifmm_ops_get_info(kifmm_ops ops, kifmm_ops_info* out) {
  return guarded([&] {
    const Ops* o = as_ops(ops);
    require(out != nullptr, "out is null");
    std::memset(out, 0, sizeof(*out));
    out->p = o->p;
    out->n_surface = o->n;
    out->rank_m2l = o->k;
    out->rank_c2e = o->kc;
    out->n_m2l_offsets = kNumOffsets;
    out->eps_pinv = o->eps_pinv;
    out->eps_svd = o->eps_svd;
    out->alpha_inner = kAlphaInner;
    out->alpha_outer = kAlphaOuter;
  });
}

kifmm_status kifmm_ops_get_matrix(kifmm_ops ops, int which, int index, double* out, int64_t capacity) {
  return guarded([&] {
    const Ops* o = as_ops(ops);
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
  return guarded([&] { release(as_ops(ops)); });
}

kifmm_status kifmm_plan_create(kifmm_tree tree, kifmm_ops ops, int nrhs, unsigned flags, int device,
                               kifmm_plan* out) {
  return guarded([&] {
    require(out != nullptr, "out is null");
    *out = nullptr;
    *out = reinterpret_cast<kifmm_plan>(create_plan(as_tree(tree), as_ops(ops), nrhs, flags, device));
  });
}

kifmm_status kifmm_evaluate(kifmm_plan plan, const float* charges, float* potential, float* gradient, void* stream) {
  return guarded([&] { evaluate_plan(as_plan(plan), charges, potential, gradient, (hipStream_t)stream); });
}

kifmm_status kifmm_evaluate_vjp(kifmm_plan plan, const float* charges, const float* weights, const float* field,
                                float* grad_charges, float* grad_points, void* stream) {
  return guarded([&] {
    evaluate_vjp(as_plan(plan), charges, weights, field, grad_charges, grad_points, (hipStream_t)stream);
  });
}

kifmm_status kifmm_plan_destroy(kifmm_plan plan) {
  return guarded([&] { release(as_plan(plan)); });
}

kifmm_status kifmm_plan_set_timing(kifmm_plan plan, int enable) {
  return guarded([&] {
    Plan* p = as_plan(plan);
    if (!enable && p->timing) p->collect_times();
    p->timing = enable != 0;
  });
}

kifmm_status kifmm_plan_get_stage_times(kifmm_plan plan, double* ms, int64_t* counts, int reset) {
  return guarded([&] {
    Plan* p = as_plan(plan);
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
    const Plan* p = as_plan(plan);
    require(stats != nullptr && count >= 0, "stats is null or count is negative");
    const int64_t form = p->m2l_pieces ? 3 : p->m2l_wide ? 2 : p->m2l_gather ? 1 : 0;
    const bool up = p->up && p->up_on;
    const int64_t stage_pairs = up ? p->m2l_pairs_leaf : p->m2l_pairs;
    const int64_t slab = form == 0 ? p->m2l_lds_ld - 4 : form == 3 ? 32 : 0;
    const int64_t threads = p->nrhs == 1 ? p->p2p_threads : 0;
    const int64_t v[12] = {p->p2p_pairs, p->m2l_pairs, p->far ? p->slots[p->L] : 0, p->m2l_targets, p->k, p->n,
                           p->nrhs, form, stage_pairs, up ? 1 : 0, slab, threads};
    for (int i = 0; i < count && i < 12; ++i) stats[i] = v[i];
  });
}

kifmm_status kifmm_plan_read_density(kifmm_plan plan, int kind, int level, float* host_out, int64_t capacity) {
  return guarded([&] { read_density(as_plan(plan), kind, level, host_out, capacity); });
}

}  // extern "C"
