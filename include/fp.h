/*
 * fp.h -- C-ABI of libfp.so: Monte Carlo frame potentials of random quantum
 * circuit ensembles on one AMD Instinct MI355X (gfx950).
 *
 * The method (Liu, Liu, Alexeev, Jiang, "Estimating the randomness of quantum
 * circuit ensembles up to 50 qubits", arXiv 2205.09900):
 *   F^(k) = E_{U,V} |Tr(U^dagger V)|^{2k}             (Sec. I.A, frame potential)
 *   F^(k) ~ (1/N) sum_i |Tr(U_i^dagger V_i)|^{2k}      (Sec. II.A, Monte Carlo)
 * with every trace an exact tensor-network contraction along the qubit
 * direction (Sec. II.A, trace as a contraction; Methods A).
 *
 * Conventions shared by every call
 *   - Every call returns int: FP_OK (0) or a negative FP_E* code, and never
 *     throws.  fp_last_error() gives a thread-local message for the last error.
 *   - Device pointers are plain HIP device addresses (e.g. torch tensors on
 *     cuda:N); `stream` is a hipStream_t passed as void* (NULL = null stream).
 *     Work is asynchronous on `stream` unless the call says otherwise.
 *   - The caller allocates and frees every buffer it passes.  The library
 *     keeps no pointer after a call returns, except for work in flight on
 *     `stream`.  Plans and tuning tables are cached inside the library.
 *   - Sampling or contracting 0 pairs is a no-op returning FP_OK.
 *   - Calls are re-entrant for distinct streams and workspaces.
 *
 * Qubits: q = 2, an open 1D chain of n qubits (2 <= n <= 64).  A two-qubit
 * gate on bond b acts on qubits (b, b+1) as a 4x4 complex matrix, row-major,
 * composite index 2*x_b + x_{b+1} (qubit b is the more significant bit),
 * rows = outputs, columns = inputs, each complex stored as (re, im).
 */
#ifndef FP_H
#define FP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
enum {
  FP_OK = 0,
  FP_EINVAL = -1,   /* bad argument: NULL pointer, n outside 2..64, depth < 1,
                       unknown ansatz or precision, num_pairs < 0, k_max outside
                       1..8, num_pairs == 0 where a mean is asked for, or a
                       buffer smaller than the call needs                      */
  FP_ETOOBIG = -2,  /* a boundary tensor exceeds the workspace or the limits  */
  FP_EDEVICE = -3,  /* a HIP runtime error (text in fp_last_error)            */
  FP_ENOTIMPL = -4, /* combination the library does not provide             */
  FP_ENUMERIC = -5  /* a non-finite trace reached the reduction               */
};

/* ---- ensembles (Results, Fig. 2) ------------------------------------------ */
enum {
  FP_BRICKWORK_HAAR = 0,    /* "parallel random unitaries": layer t = 1..depth acts
                               on bonds b = t-1 (mod 2); Haar U(4) gates          */
  FP_LOCAL_RANDOM_HAAR = 1, /* "local random unitaries": depth = steps; each step is
                               one Haar U(4) gate on a uniformly chosen bond      */
  FP_HEA_RYRZ_CZ = 2,       /* hardware-efficient ansatz: depth = layers; a layer is
                               RY(theta) then RZ(phi) on every qubit, then CZ on
                               every bond; theta, phi ~ U(0, 2 pi]                */
  FP_HEA_PAULI_CNOT = 3,    /* the paper's hardware-efficient ansatz (Fig. 2c;
                               Sec. II.C): a wall of RY(pi/4), then per layer a
                               rotation exp(-i theta P / 2) on every qubit (P
                               uniform in {X, Y, Z}, theta ~ U(0, 2 pi]) and two
                               walls of CNOT (control q, target q+1), first on
                               the bonds q even, then q odd; depth = layers     */
  FP_HEA_PAULI_CZ = 4,      /* the same with CZ walls                            */
  FP_BRICKWORK_QUDIT = 5    /* brickwork of qudits (Sec. II.A, the generalisation
                               to local dimension q > 2): n_qubits counts the
                               qudits, local_dim holds q (3, 4 or 5); layer
                               t = 1..depth acts on bonds b = t-1 (mod 2); Haar
                               U(q^2) gates, composite index q x_b + x_{b+1}.
                               Contracted in LDS, one pair per workgroup: the
                               boundary of q^(2(depth-1)) entries must fit
                               160 KiB with the gate tables (q = 3: depth <= 5;
                               q = 4: depth <= 4; q = 5: depth <= 4 in FP_C64
                               and FP_BF16X3, <= 3 in FP_C128); deeper ones
                               fail with FP_ETOOBIG                          */
};

/* ---- precisions ------------------------------------------------------------ */
enum {
  FP_C128 = 0,  /* float64 gates, complex128 boundary                           */
  FP_C64 = 1,   /* float32 gates, complex64 boundary, power-of-two rescale per
                   column with the exponent kept in float64                    */
  FP_BF16X3 = 2 /* float32 storage (gates, boundary) as FP_C64; every complex
                   multiply-add of the contraction (merged-gate products, GATE
                   ops, HEA pointwise products) takes each real product as
                   hi_a hi_b + hi_a lo_b + lo_a hi_b with x = hi + lo, hi and
                   lo bf16 (round to nearest even), float32 accumulation.
                   GATE ops on boundaries of 2^9 entries or more run on the
                   bf16 matrix cores as 16x16 blocks (two GATEs on four
                   distinct bits, formed in float32 and then split, or one
                   GATE times the identity on two further bits).
                   Expected error vs FP_C128 about 2^-16 per product; the
                   HEA one-layer case (a product of 2x2 traces in float64)
                   is the same as FP_C64                                        */
};

typedef struct {
  int32_t ansatz;    /* FP_BRICKWORK_HAAR ... FP_BRICKWORK_QUDIT                 */
  int32_t n_qubits;  /* 2..64 (qubits, or qudits for FP_BRICKWORK_QUDIT)         */
  int32_t depth;     /* layers (brickwork, HEA) or steps (local random), >= 1    */
  int32_t local_dim; /* FP_BRICKWORK_QUDIT: q in 3..5; every other ansatz: 0     */
} fp_ensemble_t;

typedef struct {
  int32_t ensemble_index; /* index into the ensemble array of the call          */
  int32_t precision;      /* FP_C64 or FP_C128                                  */
  int64_t first_pair;     /* first pair index of the group inside its gate buffer */
  int64_t num_pairs;      /* pairs in the group                                  */
} fp_group_t;

/*
 * fp_gate_bytes_per_pair -- bytes one (U, V) pair occupies in a gate buffer.
 * Layout of one pair (the pair stride is this value):
 *   Haar ensembles: [U gates][V gates], each gate 16 complex numbers (Real =
 *     double for FP_C128, float otherwise) in time order; brickwork gates are
 *     ordered layer by layer, bonds ascending inside a layer.
 *   local random: followed by [U bonds][V bonds], one int32 per step.
 *   HEA: [U angles][V angles], per layer l and qubit q the pair (theta, phi)
 *     as Real, index ((l * n) + q) * 2.
 *   Pauli-rotation HEA: the same with the pair (theta, axis), axis 0, 1, 2
 *     for X, Y, Z stored as Real (the fixed RY(pi/4) wall is not stored; it
 *     cancels inside the trace).
 *   qudit brickwork: [U gates][V gates], each gate q^2 x q^2 complex, row
 *     major, in the brickwork order of the qubit case.
 * The total is padded to a multiple of 64 bytes.  Returns 0 for an invalid
 * ensemble or precision.
 */
size_t fp_gate_bytes_per_pair(const fp_ensemble_t* ens, int precision);

/*
 * fp_sample_gates -- draw num_pairs independent (U, V) pairs of the ensemble
 * (Results, Fig. 2; Methods B for the Haar gates) into d_gates.
 * Pair i of the call is global pair first_pair + i.  Every random number
 * comes from Philox4x32-10 (Salmon et al., SC'11) with
 *   key = (seed low 32 bits, seed high 32 bits),
 *   counter = (word, item, pair low 32 bits, pair bits 32..62 | circuit << 31),
 * circuit 0 = U, 1 = V, so any split of a batch yields identical gates:
 *   Haar gate g: item g, words 0..15 -> complex Gaussian entry (w/4, w%4) by
 *     Box-Muller of U53(x0, x1), U53(x2, x3); the gate is the Q factor of the
 *     QR decomposition with a positive real diagonal in R (Mezzadri 2007).
 *     Qudit gates the same with words 0..q^4-1 -> entry (w / q^2, w % q^2).
 *   local-random step s: item s, words 16, 17, ...: first 32-bit output x with
 *     x < 2^32 - (2^32 mod (n-1)) gives the bond x mod (n-1).
 *   HEA layer l, qubit q: item l*n + q, word 0: theta = 2 pi U53(x0, x1),
 *     phi = 2 pi U53(x2, x3).
 *   Pauli-rotation HEA layer l, qubit q: item l*n + q, word 0: axis = x mod 3
 *     for the first x of (x0, x1) below 2^32 - 1 (0 if neither is),
 *     theta = 2 pi U53(x2, x3).
 *   U53(a, b) = ((a >> 5) * 2^26 + (b >> 6) + 1) * 2^-53.
 * Values are computed in float64 and stored as the precision's Real.
 * gates_bytes must be >= num_pairs * fp_gate_bytes_per_pair(ens, precision).
 * Errors: FP_EINVAL, FP_EDEVICE.
 */
int fp_sample_gates(const fp_ensemble_t* ens, int64_t num_pairs, uint64_t seed,
                    uint64_t first_pair, int precision, void* d_gates,
                    size_t gates_bytes, void* stream);

/*
 * fp_workspace_bytes -- device workspace fp_contract_trace_batch needs for
 * num_pairs pairs of this ensemble (plans of local random pairs and
 * boundaries too large for on-chip memory).  Writes *out_bytes.
 * Errors: FP_EINVAL, FP_ETOOBIG (a boundary exceeds the library limits).
 */
int fp_workspace_bytes(const fp_ensemble_t* ens, int64_t num_pairs, int precision,
                       size_t* out_bytes);

/*
 * fp_contract_trace_batch -- Tr(U_i^dagger V_i) for every pair of a gate
 * buffer laid out as fp_sample_gates writes it (Sec. II.A: the trace as a
 * tensor contraction, contracted along the qubit direction so that few
 * indices are exposed; Methods A: cost linear in n, memory exponential in
 * depth).  The network of W = U^dagger V is swept one qubit column at a time;
 * the boundary tensor after column j is indexed by the wire segments of qubit
 * j+1 that connect to both neighbouring bonds, and in FP_C64 it is rescaled
 * by a power of two after every column with the exponent kept in float64.
 * d_trace receives 2*num_pairs doubles (re, im of pair i at 2i, 2i+1).
 * Local random pairs are planned on the device (each pair's network differs)
 * and the launches that follow are derived there from the plans.  Outside
 * stream capture the call then waits for the planning of its batch (not for
 * its sweeps) to size each launch exactly, unless the last call that waited
 * for the same ensemble and precision found more than a fifth of its pairs
 * beyond 2^12 register entries; in that case, and while `stream` is being
 * captured, it does not wait, and the launches take their pairs from the
 * device's plan whatever their size (sizes from the last call that waited
 * for the same ensemble and precision).  Either way a pair that
 * cannot be contracted (its plan exceeds the planner's limits, a register
 * beyond 2^31 entries, or no room in the workspace for it) gets a NaN trace,
 * which fp_frame_potential reports as FP_ENUMERIC.  No pair is dropped.
 * Errors: FP_EINVAL, FP_ETOOBIG (workspace too small for the plans, or, for
 * fixed topologies, a boundary beyond the limits; fp_workspace_bytes reports
 * the size), FP_ENOTIMPL, FP_EDEVICE.
 */
int fp_contract_trace_batch(const fp_ensemble_t* ens, int64_t num_pairs, int precision,
                            const void* d_gates, double* d_trace, void* d_workspace,
                            size_t workspace_bytes, void* stream);

/*
 * fp_frame_potential -- the Monte Carlo estimate
 *   F^(k) = (1/N) sum_i |Tr_i|^{2k},  k = 1..k_max       (Sec. II.A)
 * and its standard error (sample standard deviation / sqrt(N)) from one
 * trace array, as the same traces serve every k (Supplementary Figures,
 * sample sizes).  d_trace: 2*num_pairs doubles on the device.  h_F receives
 * k_max doubles on the host; h_stderr (k_max doubles) may be NULL.
 * Accumulation is float64 with a fixed reduction order (bitwise
 * reproducible).  Synchronises `stream` before returning.
 * Errors: FP_EINVAL (num_pairs < 1, k_max outside 1..8, NULL), FP_ENUMERIC
 * (a non-finite trace), FP_EDEVICE.
 */
int fp_frame_potential(const double* d_trace, int64_t num_pairs, int k_max,
                       double* h_F, double* h_stderr, void* stream);

/*
 * fp_set_launch_mode -- how later fp_contract_trace_batch calls of local
 * random ensembles launch their sweeps outside stream capture (a captured
 * call never waits, whatever the mode):
 *   FP_LAUNCH_AUTO      as described at fp_contract_trace_batch (default);
 *   FP_LAUNCH_WAIT      always read the planning's set-up back first and
 *                       launch every class at its exact size;
 *   FP_LAUNCH_WAIT_FREE never wait: the launches take their pairs from the
 *                       device's set-up through counters.
 * Both modes give identical traces.  Process-wide; takes effect at the next
 * call.  Errors: FP_EINVAL (unknown mode).
 */
enum { FP_LAUNCH_AUTO = 0, FP_LAUNCH_WAIT = 1, FP_LAUNCH_WAIT_FREE = 2 };
int fp_set_launch_mode(int mode);

/*
 * fp_frame_potential_noalloc -- fp_frame_potential for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same reduction, kernels and result
 * bit for bit, with its partial results in a static scratch array of the
 * library (128 KiB per device, held until the process ends) instead of
 * memory allocated per call.  It calls no allocating routine.  Every call on
 * a device shares that device's array, so calls that overlap on one device
 * (on different streams or host threads) race and must be serialised by the
 * caller.  The reduction needs at most about 107 KiB for any num_pairs; a
 * larger need would fail with FP_ETOOBIG.  Synchronises `stream`.
 * Errors: as fp_frame_potential, FP_ETOOBIG.
 */
int fp_frame_potential_noalloc(const double* d_trace, int64_t num_pairs, int k_max,
                               double* h_F, double* h_stderr, void* stream);

/* ---- statistics of the estimates ------------------------------------------ */
/*
 * fp_haar_frame_potential -- F_Haar^(k) of U(dim): the number of
 * permutations of k elements whose longest increasing subsequence is at most
 * dim, which is k! for dim >= k (the paper's Haar value, Sec. I.A; exact for
 * every dim by the count).  k in 1..10.  Host only.  Errors: FP_EINVAL.
 */
int fp_haar_frame_potential(int k, double dim, double* out);

/*
 * fp_bootstrap -- bootstrap distribution of F^(k), k = 1..k_max
 * (Supplementary Methods, bootstrapping for uncertainty quantification; the
 * paper uses 300 resamples): resample r draws num_pairs traces with
 * replacement, draw i taking index floor(u N / 2^64) of the 64-bit word u of
 * Philox4x32-10 block i >> 1 (x0 + 2^32 x1 for even i, x2 + 2^32 x3 for odd
 * i) with counter (block low 32, block high 32, r, 0xB0075A3B) and key
 * seed, and F_r^(k) is the mean of |Tr|^{2k} over the draws (float64, terms
 * scaled by a batch power of two, fixed order).
 * d_samples (k_max x resamples doubles on the device, F_r^(k) at
 * (k-1) * resamples + r, in resample order) may be NULL.  h_median, h_lo,
 * h_hi (k_max doubles each, may be NULL) receive the median and the
 * (1 -/+ coverage)/2 quantiles (linear interpolation between order
 * statistics at q (R-1)).  resamples in 2..1024.  Synchronises `stream`.
 * Errors: FP_EINVAL, FP_ENUMERIC (a non-finite trace), FP_EDEVICE.
 */
int fp_bootstrap(const double* d_trace, int64_t num_pairs, int k_max, int resamples, uint64_t seed,
                 double* d_samples, double* h_median, double* h_lo, double* h_hi, double coverage,
                 void* stream);

/*
 * fp_layers_to_epsilon -- layers needed for an epsilon-approximate k-design
 * from estimates at several depths (main text: F - F_Haar = A^2 exp(-2l/C)
 * gives l = C (k n log q + log A + log(1/epsilon)); Supplementary Methods,
 * choice of curve fitting region: only depths with
 * 0 < (F - F_Haar)/F_Haar < rel_dev_max, the paper's 5).  d_F holds
 * n_layers x resamples doubles on the device (F of depth h_layers[j] in
 * sample r at j * resamples + r; bootstrap samples of each depth, or one
 * estimate per depth with resamples = 1); h_layers are the depths (host).
 * Per sample, a least-squares line through (l, log(F - F_Haar)) over the
 * qualifying depths; a sample with fewer than two of them, or a line that
 * does not decay, has no value (NaN in d_out, counted in *h_failed).
 * d_out (resamples doubles, device) may be NULL; *h_median is the median of
 * the samples that have a value (NaN if none).  Synchronises `stream`.
 * Errors: FP_EINVAL, FP_EDEVICE.
 */
int fp_layers_to_epsilon(const double* d_F, const int32_t* h_layers, int n_layers, int resamples, double F_haar,
                         double epsilon, int n_qubits, int q, int k, double rel_dev_max, double* d_out,
                         double* h_median, int* h_failed, void* stream);

/*
 * fp_sample_size_decision -- the adaptive sample-size rule (Supplementary
 * Methods, determination of sample sizes): FP_STOP_BUDGET once n_done >=
 * n_max or seconds >= max_seconds; else FP_CONTINUE while the estimate is
 * unphysical (F < F_haar, or F above the estimate at one layer less,
 * F_lower, when F_lower > 0); else FP_STOP_RESOLVED once F - F_haar > z se;
 * else FP_CONTINUE.  Host only.  Errors: FP_EINVAL.
 * fp_frame_potential_adaptive -- sample, contract and reduce batches of
 * batch_pairs pairs (global pairs 0, 1, ... of `seed`, as fp_sample_gates
 * numbers them) into d_trace (2 * max_pairs doubles) until the rule, applied
 * to F^(k_rule) of all pairs so far after every batch, stops; writes F^(k)
 * and its standard error, k = 1..k_max (h_stderr may be NULL), the pairs
 * used and the reason.  d_gates and d_ws hold one batch (fp_gate_bytes_per_pair
 * and fp_workspace_bytes for batch_pairs).  Synchronous.
 * Errors: as fp_contract_trace_batch and fp_frame_potential.
 */
enum { FP_CONTINUE = 0, FP_STOP_RESOLVED = 1, FP_STOP_BUDGET = 2 };
int fp_sample_size_decision(double F, double se, double F_haar, double F_lower, double z, int64_t n_done,
                            int64_t n_max, double seconds, double max_seconds, int* decision);
int fp_frame_potential_adaptive(const fp_ensemble_t* ens, int precision, int k_max, int k_rule, uint64_t seed,
                                int64_t batch_pairs, int64_t max_pairs, double max_seconds, double z, double F_haar,
                                double F_lower, void* d_gates, size_t gates_bytes, void* d_ws, size_t ws_bytes,
                                double* d_trace, double* h_F, double* h_stderr, int64_t* h_pairs_used,
                                int* h_reason, void* stream);

/* ---- uneven batches ------------------------------------------------------- */
/*
 * fp_contract_trace_groups -- contract several groups of pairs with different
 * ensembles (depths, qubit counts) in one persistent launch.  Group g reads
 * pairs [first_pair, first_pair + num_pairs) of the buffer d_gates[g]
 * (laid out for ens[groups[g].ensemble_index] at groups[g].precision) and
 * writes their traces consecutively into d_trace, in group order.  Work items
 * are ordered by their planned cost, largest first.  Tile shapes come from
 * the tuning table (fp_autotune).  d_ws / ws_bytes as for
 * fp_contract_trace_batch (fp_workspace_bytes_groups gives the size).
 * Errors: as fp_contract_trace_batch.
 */
int fp_workspace_bytes_groups(const fp_ensemble_t* ens, int n_ens, const fp_group_t* groups,
                              int n_groups, size_t* out_bytes);
int fp_contract_trace_groups(const fp_ensemble_t* ens, int n_ens, const fp_group_t* groups,
                             int n_groups, const void* const* d_gates, double* d_trace,
                             void* d_ws, size_t ws_bytes, void* stream);

/*
 * fp_autotune -- time the launch choices of the persistent sweep of
 * fp_contract_trace_groups for one fixed-topology ensemble (brickwork or
 * HEA whose register fits LDS) and precision on the current device, with
 * synthetic gates drawn by fp_sample_gates, keep the fastest in the
 * library's tuning table, and write its index to *out_choice:
 *   choice = 3 * lane_class + task_size,
 *   lane_class 0 "tiny":  16 lanes per pair, 16 pairs per workgroup;
 *              1 "small": 64 lanes per pair, 4 pairs per workgroup;
 *              2 "mid":   256 lanes, one pair per workgroup;
 *              3 "large": 1024 lanes (512 in FP_C128), one pair per workgroup;
 *              a class is a candidate only while its workgroup holds its
 *              pairs' registers in LDS;
 *   task_size 0, 1, 2: about 5e6, 2e7, 8e7 algorithmic flops per task taken
 *                 from the launch's counter.
 * fp_contract_trace_groups uses the table's entry of every group's ensemble
 * and precision, else the class the per-ensemble launch takes for the
 * register width (tiny up to 2^6 entries, small up to 2^10 (2^9 in
 * FP_C128), mid up to 2^12, large beyond) and 2e7 flops per task; it makes
 * one persistent launch per lane class and register-size bucket.  Synchronous.  Uses d_ws (ws_bytes) as scratch, which must hold
 * fp_autotune_workspace_bytes bytes (0 for an ensemble it cannot tune).
 * fp_autotune_table writes the table as text, one line per tuned key,
 *   "<arch> <ansatz> <n> <depth> <precision> tiny|small|mid|large <task flops> <ms>",
 * into buf (capacity cap, NUL-terminated); fp_autotune_load reads such text.
 * Errors: FP_EINVAL, FP_ETOOBIG (workspace), FP_ENOTIMPL (local random,
 * qudit brickworks, or a boundary beyond LDS), FP_EDEVICE.
 */
size_t fp_autotune_workspace_bytes(const fp_ensemble_t* ens, int precision);
int fp_autotune(const fp_ensemble_t* ens, int precision, void* d_ws, size_t ws_bytes,
                int* out_choice, void* stream);
int fp_autotune_table(char* buf, size_t cap);
int fp_autotune_load(const char* text);

/* ---- plan inspection (host only; no device is touched) ---------------------- */
/*
 * fp_plan_info -- plan the sweep of a fixed-topology ensemble (brickwork or
 * HEA) on the host and report, per column j = 0..n-2, log2 of the boundary
 * size after the column (out_bits, n-1 entries, may be NULL), and overall
 * the largest boundary exponent during the sweep (*peak_bits), the number of
 * complex multiply-adds of one contraction (*macs) and the number of
 * program operations (*ops).  Any output pointer may be NULL.
 * Errors: FP_EINVAL, FP_ENOTIMPL (local random ensembles are planned per pair).
 */
int fp_plan_info(const fp_ensemble_t* ens, int32_t* out_bits, int32_t* peak_bits,
                 double* macs, int64_t* ops);

/*
 * fp_plan_local_random_host -- plan one local random pair from its bond
 * lists (host arrays of `steps` int32 each) with the same planner the device
 * runs, and report as fp_plan_info.  Host only.
 */
int fp_plan_local_random_host(int n_qubits, int steps, const int32_t* bonds_u,
                              const int32_t* bonds_v, int32_t* out_bits, int32_t* peak_bits,
                              double* macs, int64_t* ops);

/*
 * fp_plan_program_host -- the register program the sweep kernels execute for
 * one pair of two-qubit-gate circuits with the given bond lists (steps gates
 * per circuit, time order).  ops receives up to max_ops records of 8 bytes
 * {uint8 type, uint8 p, uint8 q, uint8 bits; int32 arg}: type 0 = GATE on
 * register bits (p, q) with merged gate `arg`, 1 = BELL (two new top bits
 * holding a delta), 2 = TRACE over bits p < q (removed, higher bits move
 * down), 3 = end of column; `bits` is the register width after the op.
 * wgates receives (first, count) int32 pairs per merged gate and factors the
 * factor codes (code < steps: gate `code` of V; otherwise gate
 * 2*steps-1-code of U, conjugate-transposed), in time order.  *num_ops and
 * *log2_factor (a factor 2 per qubit no gate touches) are written.  Host only.
 * Errors: FP_EINVAL (bad bonds or max_ops too small), FP_ETOOBIG.
 */
int fp_plan_program_host(int n_qubits, int steps, const int32_t* bonds_u, const int32_t* bonds_v,
                         void* ops, int64_t max_ops, int32_t* wgates, int32_t* factors,
                         int64_t* num_ops, int32_t* log2_factor);

/* ---- learned control variate (extension) ------------------------------------ */
/*
 * Surrogate network for the control variate: inputs are sin and cos of every
 * angle of U and V (features = 8 * n * L for the HEA), three hidden layers of
 * width H with SiLU, one linear output, float32.  Parameters live in one
 * device buffer `d_params` of fp_mlp_param_count(n_in, H) floats, laid out
 * as W1 (n_in x H, row-major), b1 (H), W2 (H x H), b2, W3 (H x H), b3, W4 (H),
 * b4 (1).  The optimiser state d_adam holds 2 * param_count floats (m, v).
 *
 * fp_mlp_features: angles of num_pairs HEA pairs (the gate buffer of
 *   fp_sample_gates, FP_C64 layout) -> d_x (num_pairs x n_in floats).
 * fp_mlp_forward: d_y[i] = net(d_x[i]) for a batch; d_act may be NULL, or hold
 *   fp_mlp_act_floats(batch, H) floats to keep the activations for backward.
 * fp_mlp_backward: gradient of (1/batch) sum_i (y_i - t_i)^2 with respect to
 *   the parameters into d_grad (param_count floats); *h_loss gets the loss
 *   (synchronous when h_loss != NULL).
 * fp_mlp_adam_step: one Adam update (step >= 1, bias-corrected).
 * Errors: FP_EINVAL, FP_EDEVICE.
 */
int64_t fp_mlp_param_count(int n_in, int hidden);
int64_t fp_mlp_act_floats(int64_t batch, int hidden);
int fp_mlp_init(int n_in, int hidden, uint64_t seed, float* d_params, void* stream);
int fp_mlp_features(const fp_ensemble_t* ens, int64_t num_pairs, const void* d_gates,
                    float* d_x, void* stream);
int fp_mlp_forward(int n_in, int hidden, int64_t batch, const float* d_params,
                   const float* d_x, float* d_y, float* d_act, void* stream);
int fp_mlp_backward(int n_in, int hidden, int64_t batch, const float* d_params,
                    const float* d_x, const float* d_act, const float* d_target,
                    float* d_grad, double* h_loss, void* stream);
int fp_mlp_adam_step(int64_t count, float* d_params, const float* d_grad, float* d_adam,
                     int step, float lr, float beta1, float beta2, float eps, void* stream);
/*
 * fp_mlp_gemm -- the dense product the network runs on the MFMA units:
 * C (M x N, row-major, ldc) = op(A) op(B), op(A) = A (M x K, lda) or, with
 * trans_a, A^T for A stored K x M; likewise B (K x N).  float32 with float32
 * accumulation.  Errors: FP_EINVAL, FP_EDEVICE.
 */
int fp_mlp_gemm(int M, int N, int K, const float* d_A, int lda, int trans_a, const float* d_B, int ldb,
                int trans_b, float* d_C, int ldc, void* stream);

/*
 * fp_mlp_targets -- training targets t_i = scale * |Tr_i|^{2k} (float32) from a
 * device trace array (2*num_pairs doubles).  Errors: FP_EINVAL, FP_EDEVICE.
 * fp_cv_coefficient -- c = Cov(f, g) / Var(g) with f_i = |Tr_i|^{2k}, float64,
 * fixed reduction order, written to *h_c (0 when g is constant).  Meant for
 * a hold-out set disjoint from the pairs the estimate uses, so that the
 * estimator stays unbiased.  Synchronises `stream`.
 */
int fp_mlp_targets(const double* d_trace, int64_t num_pairs, int k, double scale, float* d_t, void* stream);
int fp_cv_coefficient(const double* d_trace, const float* d_g, int64_t num_pairs, int k, double* h_c,
                      void* stream);
/*
 * Log-space fitting of the surrogate (|Tr|^2 is close to a product over
 * qubits, so its logarithm is close to additive in the angles):
 * fp_log_moments -- mean and sample standard deviation (float64) of
 *   L_i = log(|Tr_i|^2 + eps) over a device trace array.  Synchronises.
 * fp_mlp_log_targets -- t_i = (L_i - mean) / std_dev as float32.
 * fp_mlp_link -- g_i = exp(k (mean + std_dev y_i) - shift) as float32: the
 *   network output y mapped back to |Tr|^{2k} in units of e^shift (the
 *   exponent is capped at 80).
 * Errors: FP_EINVAL, FP_EDEVICE.
 */
int fp_log_moments(const double* d_trace, int64_t num_pairs, double eps, double* h_mean, double* h_std,
                   void* stream);
int fp_mlp_log_targets(const double* d_trace, int64_t num_pairs, double eps, double mean, double std_dev,
                       float* d_t, void* stream);
int fp_mlp_link(const float* d_y, int64_t n, int k, double mean, double std_dev, double shift, float* d_g,
                void* stream);

/*
 * fp_cv_holdout -- statistics of a hold-out set for the control variate,
 * f_i = |Tr_i|^{2k} against surrogate values g_i (float64, fixed reduction
 * order), into h_stats[6]: c = Cov(f, g)/Var(g) (0 for constant g), the
 * correlation rho (0 if f or g is constant), mean and sample variance of f,
 * mean and sample variance of g.  Synchronises `stream`.
 * fp_moments_f32 -- mean and sample variance (float64) of a float array on
 *   the device (n >= 2).  Synchronises `stream`.
 * Errors: FP_EINVAL, FP_ENUMERIC (non-finite statistics), FP_EDEVICE.
 */
int fp_cv_holdout(const double* d_trace, const float* d_g, int64_t num_pairs, int k, double* h_stats,
                  void* stream);
int fp_moments_f32(const float* d_x, int64_t n, double* h_mean, double* h_var, void* stream);
/*
 * fp_cv_choose -- the rule that keeps the control variate or falls back to
 * the plain estimator, decided before the estimation pairs are drawn (so it
 * cannot bias the estimate): with correlation rho between f and g and costs
 * of sec_per_exact per exact pair and sec_per_surrogate per surrogate draw,
 * the best split of a time budget gives a variance proportional to
 *   (sqrt((1 - rho^2) sec_per_exact) + |rho| sqrt(sec_per_surrogate))^2,
 * against sec_per_exact for the plain mean.  *time_ratio (may be NULL)
 * receives the ratio of the two; *use_cv = 1 when it is below 1.  Host only.
 * fp_cv_time_to_rel_se -- wall time to reach a relative standard error
 * rel_se on F, from stats_B (fp_cv_holdout of the exact pairs against their
 * surrogate values; F = their mean of f), the coefficient c in use and the
 * variance var_g_C of the surrogate draws: plain var_f / (rel_se F)^2 x
 * sec_per_exact; control variate (sqrt(var_r sec_per_exact) +
 * |c| sqrt(var_g_C sec_per_surrogate))^2 / (rel_se F)^2, with
 * var_r = var_f - 2 c Cov(f, g) + c^2 var_g the variance of f - c g.
 * Host only.
 * Errors: FP_EINVAL.
 */
int fp_cv_choose(double rho, double sec_per_exact, double sec_per_surrogate, int* use_cv, double* time_ratio);
int fp_cv_time_to_rel_se(const double* stats_B, double c, double var_g_C, double rel_se, double sec_per_exact,
                         double sec_per_surrogate, double* t_plain, double* t_cv);

/*
 * fp_frame_potential_cv -- control-variate estimate of F^(k):
 *   F_CV = mean_B(f - c g) + c mean_C(g),  f_i = |Tr_i|^{2k}
 * over nB exact traces d_trace_B with surrogate values d_g_B, and nC fresh
 * surrogate values d_g_C; stderr^2 = Var_B(f - c g)/nB + c^2 Var_C(g)/nC.
 * With c = 0 this is the plain estimator of fp_frame_potential on B.
 * Synchronises `stream`.  Errors: FP_EINVAL, FP_ENUMERIC, FP_EDEVICE.
 */
int fp_frame_potential_cv(const double* d_trace_B, const float* d_g_B, int64_t nB,
                          const float* d_g_C, int64_t nC, int k, double c, double* h_F,
                          double* h_stderr, void* stream);

/* ---- measurement ----------------------------------------------------------- */
/*
 * fp_profile_begin / fp_profile_end -- while enabled, every kernel launch of
 * fp_sample_gates and fp_contract_trace_batch (sampling, planning, matrix
 * preparation, sweeps) is bracketed by HIP events on its stream.
 * fp_profile_end disables timing, waits for the recorded events and writes,
 * per launch class, the summed kernel time in milliseconds, the number of
 * launches, the algorithmic flops and the algorithmic bytes.  Classes:
 *   0..3  sweeps with the boundary in LDS (local random: registers up to
 *         2^8 and 2^10 entries with one wavefront per pair, up to 2^12 and
 *         2^14 with 256 and 1024 lanes per pair; fixed topologies: 16, 64,
 *         256, 1024 lanes per pair);
 *   4     boundaries in HBM;          5  HEA transform sweep;
 *   6     local random planning;      7  GATE matrix preparation;
 *   8     gate sampling.
 * Flops: 8 real flops per complex multiply-add of the plan; for the HEA sweep
 * 2 per complex addition of the transforms and 6 per pointwise product; 0 for
 * classes 6..8.  Bytes: for classes 6..8 the data each launch must read and
 * write (bond lists and plans; gates and matrices; gates); 0 otherwise.
 * Each output array has FP_PROFILE_CLASSES entries and may be NULL.
 * Not re-entrant.
 */
#define FP_PROFILE_CLASSES 9
int fp_profile_begin(void);
int fp_profile_end(double* kernel_ms, int64_t* launches, double* flops, double* bytes);

/* ---- misc ---------------------------------------------------------------- */
const char* fp_last_error(void);
int fp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FP_H */
