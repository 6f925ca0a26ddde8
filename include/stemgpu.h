/*
 * stemgpu: contraction of a sliced stem network on one MI355X (gfx950).
 *
 * The method (paper §3, §4, §A.1-§A.3): a tensor network whose every bond has
 * dimension 2 is contracted along a "stem", one large tensor that absorbs
 * small pre-computed branch tensors one after another (§A.2 stems and
 * branches, §A.3 branch pre-computation).  A set of "sliced" labels E_s is
 * enumerated outside the contraction: each assignment of E_s (a slice)
 * selects a sub-network, and the value of the whole network is the sum of
 * the sub-network values over all slices (§A.1, slicing; the scheme
 * (E_s, T)).  A batch of amplitudes is obtained by leaving some output
 * labels open and fixing the others ("projected" labels, §3: a batch of
 * amplitudes whose closed qubits share one assignment).
 *
 * Every function returns a stem_status (0 = success).  No C++ exception
 * crosses this interface.  On failure stem_last_error() returns a message
 * (thread-local; valid until the next call on the same thread).
 *
 * Memory conventions.  A complex number is two consecutive values (real,
 * imaginary).  A tensor of rank r over a label list L is stored as 2^r
 * complex numbers in C order: label L[0] is the most significant bit of
 * the entry index.  "Device" pointers are HIP device allocations on the
 * current device; "host" pointers are ordinary host memory.  A stream
 * argument is a hipStream_t passed as void* (NULL = the null stream).
 */
#ifndef STEMGPU_H
#define STEMGPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t stem_status;

enum {
  STEM_OK = 0,
  STEM_EINVAL = 1,        /* null pointer, negative size, inconsistent descriptor */
  STEM_ELABEL = 2,        /* a label occurs in a number of tensors the method does not allow */
  STEM_ESHAPE = 3,        /* a rank exceeds the plan's limit */
  STEM_EUNSUPPORTED = 4,  /* a valid network the library does not handle yet */
  STEM_ENOMEM = 5,        /* workspace too small, or a device allocation failed */
  STEM_ERANGE = 6,        /* slice range or projected assignment out of range */
  STEM_EHIP = 7           /* a HIP runtime call failed; the message names it */
};

/* Arithmetic of the complex matrix products of the stem steps. */
enum {
  STEM_FP32 = 0,          /* FP32 inputs, FP32 MFMA products, FP32 accumulation */
  STEM_SPLIT_FP16 = 1,    /* three-term FP16 split of both factors, FP32 accumulation */
  STEM_SPLIT_BF16 = 2     /* three-term BF16 split of both factors, FP32 accumulation */
};

/* Flags of stem_contract. */
enum {
  STEM_ACCUMULATE = 1,    /* add the range's sum to out instead of overwriting it */
  STEM_TIME_STEPS = 2     /* time every kernel of the range's last slice (hipEvents);
                             read back with stem_step_info after the stream syncs */
};

/*
 * A sliced stem network (paper §A.1: the slicing scheme (E_s, T) restricted
 * to a stem-shaped tree T, §A.2).  Labels are arbitrary non-negative int32
 * values; every bond has dimension 2 (§A.1).
 *
 * Label rules checked by stem_plan_validate / stem_plan_create:
 *  - an open label occurs in at least one tensor;
 *  - a sliced or projected label is not open; it may occur in no tensor (the
 *    two halves of a join list the same ones): then every slice's value is
 *    independent of its bit;
 *  - every other label occurs in at least two tensors (more than two: a
 *    hyperedge, §A.1);
 *  - a step keeps at most 4 of the labels the stem shares with its branch
 *    (STEM_EUNSUPPORTED otherwise);
 *  - after the last branch the stem carries exactly the open labels.
 * Step i contracts the stem with branch i over the labels they share (after
 * the sliced and projected labels are fixed), which is one pairwise
 * contraction of §A.1 with time 2^|E_AB| and space 2^|E*_AB|.  A shared
 * label that a later branch or the result still carries is kept, not
 * summed (a batch label: the step is a batched product, one product per
 * assignment of its batch labels, each with its own branch sub-matrix).
 */
typedef struct stem_plan_desc {
  int32_t n_open;
  const int32_t* open_labels;     /* host; result index order, first = most significant */
  int32_t n_sliced;
  const int32_t* sliced_labels;   /* host; slice id bit (n_sliced-1-j) is the value of label j */
  int32_t n_proj;
  const int32_t* proj_labels;     /* host; projected assignment bit (n_proj-1-j) = label j */
  int32_t stem_rank;
  const int32_t* stem_labels;     /* host; labels of the initial stem, C order */
  const float* stem_data;         /* 2^stem_rank complex64, host or device (below) */
  int32_t stem_on_device;         /* nonzero: stem_data is a device pointer */
  int32_t n_branches;
  const int32_t* branch_ranks;    /* host; [n_branches] */
  const int32_t* branch_labels;   /* host; every branch's labels, concatenated */
  const float* branch_data;       /* host; every branch's 2^rank complex64, concatenated */
  int32_t precision;              /* STEM_FP32, STEM_SPLIT_FP16 or STEM_SPLIT_BF16 */
  int32_t max_rank;               /* largest allowed stem rank; 0 = 33 */
} stem_plan_desc;

/* Shape and cost of one stem step (paper §A.1: time 2^|E_AB| complex
 * multiply-adds; one complex multiply-add = 8 real floating-point ops). */
typedef struct stem_step_info {
  int32_t rank_in;        /* stem rank before the step (sliced/projected labels removed) */
  int32_t rank_out;       /* stem rank after the step */
  int32_t n_shared;       /* s: labels summed in this step, K = 2^s */
  int32_t n_free;         /* f: new labels from the branch, N = 2^f */
  int32_t permuted;       /* 1 if a stem permute runs before the product */
  int32_t last_slices;    /* slices covered by the timed launches below (0: none) */
  int64_t M, K, N;        /* product [M x K] . [K x N] -> [M x N], complex, per batch index */
  double flops;           /* 8 M K N 2^n_batch */
  double bytes;           /* 8 (M K + M N + K N) 2^n_batch: one read of stem and branch, one write */
  double perm_bytes;      /* 16 * 2^rank_in if permuted, else 0 */
  float last_gemm_us;     /* product launch of the last STEM_TIME_STEPS call, or -1;
                             one launch covers last_slices slices */
  float last_perm_us;     /* idem for the permute, or -1 */
  int32_t amode;          /* product read mode: 0 K-low, 1 M-fast */
  int32_t cmode;          /* product write mode: 0 N-fast, 1 fastest row labels kept */
  int32_t sched_tm;       /* launch schedule in use (0 = default): row blocks per wave */
  int32_t sched_ntw;      /* column tiles per workgroup */
  int32_t sched_blocks;   /* target workgroups per launch */
  int32_t sched_lds;      /* branch in LDS: 1 up to 160 KB, 0 never, -1 up to 64 KB; with
                             sched_algo 1, -1 and 0 also load the next k chunk's fragments
                             into registers ahead, 1 reads them from LDS where used; 2 (algo
                             1 or a split precision) is 1 with 8-wave workgroups, two waves
                             per SIMD sharing the copy; 3 (algo 1) keeps them in LDS up to
                             160 KB, loads them ahead, 8-wave workgroups */
  float tuned_us;         /* stem_tune's time of that schedule per launch, or -1 */
  int32_t tuned_slices;   /* slices per launch stem_tune measured with */
  int32_t n_batch;        /* labels the stem and the branch share and keep (a later branch
                             or the result carries them): the product is batched over their
                             2^n_batch values, each with its own branch sub-matrix */
  int32_t sched_algo;     /* FP32 product arithmetic: 0 real embedding (4 real products per
                             complex one), 1 the 3M method (3 real products; sched_ntw then
                             counts 16-complex-column tiles) */
} stem_step_info;

/* Summary of a plan, computed on the host without a GPU. */
typedef struct stem_plan_summary {
  int32_t n_steps;
  int32_t peak_rank;      /* largest stem rank over the steps, initial stem included */
  int32_t n_permutes;     /* steps that need a stem permute */
  int32_t n_open;
  double flops_per_slice; /* sum of the steps' flops */
  double bytes_per_slice; /* sum of the steps' algorithmic bytes */
  double perm_bytes_per_slice;
  uint64_t n_slices;      /* 2^n_sliced */
} stem_plan_summary;

typedef struct stem_plan_s* stem_plan_t;

/* Check a descriptor and compute the step shapes on the host; no device
 * memory is touched, so this runs without a GPU.  `summary` may be NULL. */
stem_status stem_plan_validate(const stem_plan_desc* desc, stem_plan_summary* summary);

/* Build a plan: validate, choose the stem's label order before every step
 * (a permute is planned only where the summed labels are not already the
 * fastest-varying ones), copy the initial stem and the branches to device
 * memory owned by the plan (sliced and projected labels moved to the most
 * significant positions, so each slice's operands are contiguous blocks),
 * and lay the branches out for the matrix-core kernels.  Host data may be
 * freed when this returns.  Uses `stream` for the device copies and
 * synchronises it before returning. */
stem_status stem_plan_create(const stem_plan_desc* desc, void* stream, stem_plan_t* plan);

/* Release the plan's device memory.  NULL is accepted. */
stem_status stem_plan_destroy(stem_plan_t plan);

stem_status stem_plan_summary_get(stem_plan_t plan, stem_plan_summary* summary);

/* Bytes of device workspace stem_contract needs to keep `slices_in_flight`
 * slices in flight (1..4096): two stem buffers of the peak size per slice.
 * The caller allocates it (any 256-byte-aligned device memory);
 * stem_contract runs as many slices per launch as the workspace it is
 * given holds. */
stem_status stem_plan_workspace_bytes(stem_plan_t plan, uint32_t slices_in_flight,
                                      uint64_t* bytes);

stem_status stem_step_info_get(stem_plan_t plan, int32_t step, stem_step_info* info);

/*
 * Contract slices [s0, s1) for n_batch projected assignments and sum them
 * (paper §A.1, slicing: the network value is the sum of the sub-network
 * values over the assignments of E_s).
 *   proj_assign: host, n_batch values in [0, 2^n_proj); NULL means one
 *                assignment 0 for every batch entry.
 *   out:         device complex128 [n_batch][2^n_open], entry order = the
 *                plan's open_labels (first most significant).  Overwritten
 *                with the sum, or added to with STEM_ACCUMULATE.  Each slice
 *                is added in FP64 in increasing slice order, one addition
 *                at a time, whatever the group size (deterministic).
 * The slices run in groups of as many as the workspace holds, each step of
 * a group in one kernel launch per kernel.  Asynchronous on `stream`; the
 * plan must not be used on two streams at once.  An empty range writes
 * zeros (or adds nothing).  s1 > 2^n_sliced or s0 > s1: STEM_ERANGE.
 * ws_bytes below stem_plan_workspace_bytes(plan, 1): STEM_ENOMEM.
 */
stem_status stem_contract(stem_plan_t plan, uint64_t s0, uint64_t s1,
                          const uint64_t* proj_assign, uint32_t n_batch,
                          void* ws, uint64_t ws_bytes, double* out,
                          uint32_t flags, void* stream);

/*
 * Autotuner of the product kernels' launch schedules (rows per wave, column
 * tiles per workgroup, workgroups per launch, branch in LDS or not).  For
 * every step it times each candidate schedule with hipEvents at
 * `slices_in_flight` slices per launch (reps launches each, after one
 * untimed launch) on the caller's workspace (ws_bytes >=
 * stem_plan_workspace_bytes(plan, slices_in_flight)), keeps the fastest in
 * the plan (used by later stem_contract calls) and appends one text line
 * per measurement to `cache_path` (NULL: no file):
 *   stem-tune-v1 <precision> <amode> <cmode> <log2 M> <log2 K> <log2 N>
 *                <slices> <tm> <ntw> <blocks> <lds> <microseconds>
 * A step whose key (precision .. slices) already has lines in the file
 * takes the fastest recorded schedule without measuring, unless reps < 0
 * (then |reps| launches are timed and the file only gains lines).  The
 * workspace contents are overwritten.  Synchronises `stream`.
 */
stem_status stem_tune(stem_plan_t plan, uint32_t slices_in_flight, void* ws, uint64_t ws_bytes,
                      int32_t reps, const char* cache_path, void* stream);

/*
 * Many slice ranges, of one or several plans (different circuits), as one
 * HIP graph launched with one call (paper §A.1: slices are independent
 * subtasks; running many at once fills the GPU when each stem is small).
 * stem_batch_create records, for plan j, the stem_contract work of slices
 * [s0[j], s1[j]) with projected assignment proj[j] (NULL: all 0) into
 * out[j] (device complex128 [2^n_open of plan j]) on a stream of its own,
 * all forked from and joined back to a private recording stream (nothing
 * is enqueued on `stream`, which is unused here and may be the null
 * stream), and instantiates the graph.
 * The workspace (device, ws_bytes) is split into n equal 256-byte-aligned
 * parts, one per plan; each must hold at least one slice of its plan
 * (else STEM_ENOMEM).  flags: STEM_ACCUMULATE as for stem_contract;
 * STEM_TIME_STEPS is not allowed (STEM_EINVAL).  Nothing runs until
 * stem_batch_launch, which may be called any number of times; each launch
 * recomputes out[j] from the plans' current device data (or adds to it
 * with STEM_ACCUMULATE).  Plans, workspace and outputs must outlive the
 * batch; a plan must not be used by two launches that overlap in time.
 */
typedef struct stem_batch_s* stem_batch_t;

stem_status stem_batch_create(int32_t n, const stem_plan_t* plans, const uint64_t* s0,
                              const uint64_t* s1, const uint64_t* proj, double* const* out,
                              void* ws, uint64_t ws_bytes, uint32_t flags, void* stream,
                              stem_batch_t* batch);
stem_status stem_batch_launch(stem_batch_t batch, void* stream);
stem_status stem_batch_destroy(stem_batch_t batch);

/*
 * Set the launch schedule of step `step` (what stem_tune would pick; paper
 * §A.3 on the GPU efficiency of small products): tm row blocks per wave (1,
 * 2, 4), ntw column tiles per workgroup (1, 2, 4, 8; with algo 1: 1, 2, 4
 * tiles of 16 complex columns), blocks target workgroups (256 .. 65536),
 * lds (-1, 0, 1; 2 with algo 1 or a split precision; 3 with algo 1; as
 * sched_lds), algo (0 or 1, as sched_algo).  Values the
 * step's shape cannot use are clamped the way the kernels clamp them
 * (read back with stem_step_info_get).  STEM_ERANGE for values outside
 * those sets; STEM_EUNSUPPORTED for algo 1 on a split-precision plan or a
 * step whose product is not whole 16-column tiles, 8-value k chunks and
 * 64-row blocks in block order.  Results are the same for every schedule
 * up to the rounding of the arithmetic chosen.
 */
stem_status stem_step_sched_set(stem_plan_t plan, int32_t step, int32_t tm, int32_t ntw,
                                int32_t blocks, int32_t lds, int32_t algo);

/*
 * Two-sided stems (paper §A.2: a contraction tree whose root joins two
 * stems).  The left and right plans are two stem networks over the same
 * sliced and projected label lists (same order); for every slice id and
 * projected assignment each is contracted as by stem_contract, and their
 * final tensors are contracted with each other over the labels open in
 * both (summed; complex products accumulated in FP64).  The join's open
 * labels are the labels open in exactly one of the plans, listed in any
 * order (open_labels, host, C order of the result, first = most
 * significant), at most 12 of them (STEM_EUNSUPPORTED); another set is
 * STEM_ELABEL, as are different sliced or projected lists.  The plans must
 * live on the same device and outlive the join; they may be the same plan.
 *
 * stem_join_contract: out (device complex128 [n_batch][2^n_open]) receives,
 * per projected assignment, the sum over slices [s0, s1) of the joined
 * value, added slice by slice in slice order (STEM_ACCUMULATE adds to out;
 * STEM_TIME_STEPS is STEM_EINVAL).  ws/ws_bytes: device workspace of at
 * least stem_join_workspace_bytes(join, 1); the number of slices per
 * launch is ws_bytes / that size (at most 4096), and the result does not
 * depend on it.  Errors as for stem_contract.  A join must not be used by
 * two calls that overlap in time, nor overlap a call on either plan.
 */
typedef struct stem_join_s* stem_join_t;

stem_status stem_join_create(stem_plan_t left, stem_plan_t right, int32_t n_open,
                             const int32_t* open_labels, stem_join_t* join);
stem_status stem_join_workspace_bytes(stem_join_t join, uint32_t slices_in_flight,
                                      uint64_t* bytes);
stem_status stem_join_contract(stem_join_t join, uint64_t s0, uint64_t s1,
                               const uint64_t* proj_assign, uint32_t n_batch, void* ws,
                               uint64_t ws_bytes, double* out, uint32_t flags, void* stream);
stem_status stem_join_destroy(stem_join_t join);

/*
 * Step shapes of a descriptor, on the host without a GPU (the same layout
 * decisions stem_plan_create makes; timing and schedule fields are -1/0).
 * Writes min(*n_steps, capacity) entries; *n_steps receives the count.
 */
stem_status stem_plan_steps(const stem_plan_desc* desc, stem_step_info* steps, int32_t capacity,
                            int32_t* n_steps);

/* ---- runtime models (ranking candidate slicing sets and stem orders) ----
 *
 * Analytic model (paper §A.1 cost with a roofline per step): a product
 * launch over g slices takes max(g 8 (MK+MN+KN) / hbm, g 8 MKN / peak) +
 * launch, a permute g 16 2^rank / hbm + launch; peak is the precision's
 * matrix rate (split paths do 3 products on the FP16/BF16 rate).  The
 * result is seconds for all 2^n_sliced slices in groups of g.
 */
typedef struct stem_hw {
  double hbm_bytes_per_s;     /* e.g. 8e12 */
  double fp32_flops_per_s;    /* dense FP32 matrix rate, e.g. 157.3e12 */
  double fp16_flops_per_s;    /* dense FP16/BF16 matrix rate, e.g. 2.5e15 */
  double launch_s;            /* per kernel launch, e.g. 4e-6 */
} stem_hw;

stem_status stem_cost_analytic(const stem_step_info* steps, int32_t n_steps, int32_t precision,
                               uint32_t slices_in_flight, uint64_t n_slices, const stem_hw* hw,
                               double* seconds);

/* Number of features of one step and the features themselves (host):
 * log2 M, log2 K, log2 N, log2 slices per launch, amode, cmode, FP32,
 * split FP16, split BF16, log2 algorithmic bytes per launch, log2 flops per
 * launch, log2 analytic seconds per launch (default stem_hw). */
#define STEM_N_FEATURES 12
stem_status stem_step_features(const stem_step_info* step, int32_t precision,
                               uint32_t slices_in_flight, float* features);

/*
 * Learned runtime model: y = W3^T relu(W2^T relu(W1^T x' + b1) + b2) + b3
 * on standardised features x' = (x - mean) * inv_std, predicting the
 * standardised log time (y t_std + t_mean = ln microseconds).  FP32, all
 * arithmetic in HIP kernels; training minimises the mean squared error with
 * full-batch Adam (Kingma and Ba 2015).  Parameters are packed as W1
 * [F x H] row-major, b1 [H], W2 [H x H], b2 [H], W3 [H], b3 [1]; their
 * initial values are inputs (host), so a caller's seeded initialisation is
 * reproduced exactly.  Buffers x (n x F), t (n) and y (n) are device FP32.
 */
typedef struct stem_mlp_s* stem_mlp_t;

int64_t stem_mlp_n_params(int32_t n_features, int32_t hidden);
stem_status stem_mlp_create(int32_t n_features, int32_t hidden, const float* init_params,
                            stem_mlp_t* mlp);
stem_status stem_mlp_set_scaling(stem_mlp_t mlp, const float* x_mean, const float* x_inv_std,
                                 float t_mean, float t_std);
stem_status stem_mlp_get_params(stem_mlp_t mlp, float* params_host);
/* Loss (device float[1]) and its gradient (device, packed like the
 * parameters) on standardised targets t' = (t - t_mean) / t_std. */
stem_status stem_mlp_loss_grad(stem_mlp_t mlp, const float* x, const float* t, int32_t n,
                               float* loss, float* grad, void* stream);
/* `steps` Adam updates (lr, beta1 0.9, beta2 0.999, eps 1e-8); loss after
 * the last one into loss (device float[1], may be NULL). */
stem_status stem_mlp_train(stem_mlp_t mlp, const float* x, const float* t, int32_t n,
                           int32_t steps, float lr, float* loss, void* stream);
/* y = predicted ln microseconds. */
stem_status stem_mlp_predict(stem_mlp_t mlp, const float* x, int32_t n, float* y, void* stream);
stem_status stem_mlp_destroy(stem_mlp_t mlp);

/*
 * Ceiling microbenchmarks (asynchronous on `stream`; time them with events).
 * stem_mb_copy: grid-stride copy of `bytes` from src to dst (device), one
 *   vec_bytes (8 or 16) access per lane per iteration, `blocks` workgroups
 *   of 256 threads; vec_bytes 64 = four 16-byte loads in flight per lane,
 *   65 = the same with non-temporal loads and stores.
 * stem_mb_mfma: `blocks` workgroups of 256 threads; every wave issues
 *   8 x iters independent MFMAs of one kind: 0 = f32 16x16x4 (2048 flops),
 *   1 = f16 16x16x32, 2 = bf16 16x16x32 (16384 flops each); out (device,
 *   blocks * 256 floats) receives a checksum so nothing is folded away.
 */
stem_status stem_mb_copy(const void* src, void* dst, uint64_t bytes, int32_t vec_bytes,
                         int32_t blocks, void* stream);
stem_status stem_mb_mfma(int32_t kind, int64_t iters, int32_t blocks, float* out, void* stream);

/*
 * Fill dst (device, n complex64) with the counter-based test tensor: entry i
 * takes SplitMix64 outputs 4i..4i+3 of stream `seed` (Steele, Lea and Flood,
 * OOPSLA 2014); each 64-bit output gives two 22-bit integers (bits 42-63 and
 * 10-31); re = (sum of the four integers of outputs 4i, 4i+1) - 2^23, im
 * likewise from 4i+2, 4i+3; both times 2^-scale_log2 (exact in FP32).
 */
stem_status stem_fill_counter(float* dst, uint64_t n, uint64_t seed, int32_t scale_log2,
                              void* stream);

/*
 * Linear cross-entropy fidelity (paper §2): out[0] = 2^n_qubits * mean |a|^2 - 1
 * over the n amplitudes, and out[1] = sum |a|^2; both in FP64.  amps: device
 * complex128 [n]; out: device double[2].  Deterministic reduction order.
 */
stem_status stem_xeb_f64(const double* amps, uint64_t n, int32_t n_qubits, double* out,
                         void* stream);

const char* stem_status_str(stem_status status);
const char* stem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STEMGPU_H */
