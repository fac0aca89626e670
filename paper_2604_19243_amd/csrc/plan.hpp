// Device plan of the kiFMM evaluate (plan.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace kifmm {

struct Plan : Object {
  Tree* tree = nullptr;
  Ops* ops = nullptr;
  unsigned flags = 0;
  int nrhs = 1;                          // right-hand sides per evaluate
  int device = 0;
  int L = 0;
  int64_t N = 0;
  bool far = false;
  int n = 0, nst = 0, k = 0, kst = 0, kc = 0, kcst = 0;
  std::vector<int64_t> slots, base, keys_per_level;
  std::vector<std::vector<int>> slot_of;
  int64_t total_slots = 0, n_leaves = 0;
  int64_t p2p_pairs = 0, m2l_pairs = 0, m2l_targets = 0;
  int m2l_rb = 0, core_rows = 0, n_items = 0, m2l_lds_ld = 0;
  int n_items_leaf = 0;                  // the first n_items_leaf items target the leaf level
  int64_t m2l_pairs_leaf = 0;            // V-list pairs with a leaf-level target

  std::vector<void*> owned;  // device allocations
  float4* d_pts = nullptr;
  int* d_order = nullptr;
  int* d_start = nullptr;
  int* d_leaves = nullptr;
  float4* d_centers = nullptr;
  int* d_blk = nullptr;
  int64_t n_groups = 0;
  int p2p_cap = 0;
  int group_slots = 8;
  float* d_surf = nullptr;
  float *d_q = nullptr, *d_t = nullptr, *d_u = nullptr, *d_d = nullptr, *d_uhat = nullptr, *d_chat = nullptr;
  float* d_zero = nullptr;
  float *d_f1 = nullptr, *d_f2 = nullptr, *d_m2m = nullptr, *d_vt = nullptr, *d_post = nullptr, *d_l2l = nullptr;
  float* d_cores = nullptr;
  int m2l_pieces = 0;                    // bfloat16 pieces per M2L operand (0: plain FP32)
  uint16_t* d_cores_b = nullptr;         // split-bfloat16 cores (lane order, all pieces)
  size_t core_stride16 = 0;              // one offset's split cores, 16-byte units
  uint16_t* d_cores_b3 = nullptr;        // three-piece cores for the levels above the leaves of a two-piece plan
  size_t core_stride16_3 = 0;
  std::vector<int*> d_nbslot;
  int* d_nonempty = nullptr;             // global slots of all non-empty boxes, levels 2..L
  int n_nonempty = 0;
  float* d_chat_part = nullptr;
  int* d_pair_offs = nullptr;
  int* d_tgt_blk = nullptr;
  int* d_src_blk = nullptr;
  M2LItem* d_items = nullptr;

  // Stage timing: a ring of event pairs per call, read back only when full or
  // on request, so timed evaluates never wait on the host.
  static constexpr int kRing = 128;
  hipStream_t side = nullptr;            // ULI stream (default priority)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipStream_t up = nullptr;              // levels above the leaves: U2U, compression, VLI, downward pass (default priority)
  bool up_on = true;                     // use it (timed against not using it at plan creation)
  int p2p_threads = kP2PMaxThreads;      // leaf-kernel workgroup size (timed against 256 at plan creation)
  double tune_ms[2][2] = {};             // evaluate [without / with the second stream][256 / 320 leaf threads] (ms)
  bool leaf_queue = false;               // one-RHS leaf sums as the persistent work-queue kernel
  double leaf_tune_ms[2] = {0.0, 0.0};   // leaf sums timed at plan creation: per-parent kernels, work queue (ms)
  int4* d_tiles = nullptr;               // work-queue tiles (leaf slot, first point, count <= 64, 0), longest first
  int n_tiles = 0;
  int* d_queue = nullptr;                // work-queue counter (cleared by a kernel before each use)
  int queue_per_cu = 8;                  // workgroups of the persistent leaf kernel per CU
  int n_cus = 1;                         // compute units of the plan's device
  double slab_tune_ms[4] = {0, 0, 0, 0}; // blocked FP32 M2L timed with 24, 32, 40, 48 k per LDS slab (ms)
  bool tuned_from_cache = false;         // the timed choices came from an earlier plan of the same shape
  bool want_up = false, want_side = false;  // the plan has the second stream / the U-list stream
  bool on_device = false;                // device resources were created (the destructor releases them)
  hipEvent_t ev_up0 = nullptr, ev_up1 = nullptr;
  float4* d_near = nullptr;              // ULI result in sorted order (phi, grad)
  bool m2l_wide = false;                 // nrhs = 32, FP32: per-target V lists with the right-hand sides as columns
  bool m2l_gather = false;               // one right-hand side, FP32: gathered form (targets as columns)
  int* d_gent_core = nullptr;            // gathered form: core index per entry
  int* d_gent_src = nullptr;             //   32 source rows of uhat per entry (zero row = total_slots)
  int* d_gtgt = nullptr;                 //   32 target slots per group (-1 = none)
  int4* d_gunits = nullptr;              //   (group, row block, first entry, end entry)
  int n_gunits = 0, n_gunits_leaf = 0;   //   the first n_gunits_leaf units target the leaf level
  double m2l_tune_ms[2] = {0.0, 0.0};    // autotuned M2L forms: blocked, gathered (ms per launch)
  int4* d_wents = nullptr;               // wide M2L: V-list entries of target pairs (core, src0 or -1, src1 or -1, 0)
  int64_t n_wide_entries = 0;
  int4* d_units = nullptr;               // wide: two per unit (see launch_m2l_wide); gathered: (group, row block, first, end)
  int n_units = 0;
  float* d_qs = nullptr;                 // nrhs > 1: sorted charges [N][nrhs]
  int4* d_tasks = nullptr;               // nrhs > 1: leaf tasks (slot, first point in the leaf, count <= 64 or 32, 0)
  int n_tasks = 0;
  float* d_vjp_fs = nullptr;             // KIFMM_VJP: grad f of the charges, [n][3], input order
  float* d_vjp_fw = nullptr;             // KIFMM_VJP: grad f of the weights, [n][3], input order

  bool timing = false;
  std::vector<hipEvent_t> ev;            // [kRing][KIFMM_N_STAGES][2]
  std::vector<unsigned char> recorded;   // [kRing][KIFMM_N_STAGES]
  int ring_used = 0, ring_slot = -1;
  double stage_ms[KIFMM_N_STAGES] = {};
  int64_t stage_count[KIFMM_N_STAGES] = {};

  ~Plan() override;
  void set_timing(bool on);
  void timing_begin_call();
  void stage_begin(int s, hipStream_t st);
  void stage_end(int s, hipStream_t st);
  void collect_times();
};

Tree* build_tree_device(const float* xyz, int64_t n, int depth, const double* cube, hipStream_t st);
Plan* create_plan(Tree* tree, Ops* ops, int nrhs, unsigned flags, hipStream_t st);
int64_t plan_workspace_bytes(Tree* tree, Ops* ops, int nrhs, unsigned flags);
void plan_stats(const Plan* plan, int64_t* v);  // KIFMM_N_STATS entries
int64_t device_memory_limit();                  // 0: none (kifmm_set_device_memory_limit)
void evaluate_plan(Plan* plan, const float* charges, float* pot, float* grad, hipStream_t st);
bool launch_m2l_form(Plan* plan, hipStream_t st, int part);
void evaluate_vjp(Plan* plan, const float* charges, const float* weights, const float* field, float* grad_charges,
                  float* grad_points, hipStream_t st);
// The same as evaluate_vjp with the two fields in the library's static device
// workspace (no allocation; needs no KIFMM_VJP).
void evaluate_vjp_noalloc(Plan* plan, const float* charges, const float* weights, const float* field,
                          float* grad_charges, float* grad_points, hipStream_t st);
void read_density(Plan* plan, int kind, int level, float* out, int64_t capacity);

}  // namespace kifmm
