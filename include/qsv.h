/*
 * qsv.h - state-vector sweep for random lattice ("supremacy") circuits on
 * AMD Instinct MI355X (gfx950).
 *
 * The library applies the gates of a random 2D-lattice circuit to a 2^n
 * complex64 amplitude vector held in device memory.  Everything below is
 * plain C: pointers, sizes and status codes.  Device buffers are owned by
 * the caller; every call that launches work is asynchronous on the HIP
 * stream passed as `stream` (a hipStream_t; NULL = the default stream).
 *
 * Conventions shared by every entry point
 *  - State layout (Section 2, preliminaries): amplitude alpha_i is stored at
 *    index i as interleaved (re, im) float32, 8 bytes; qubit k is index bit k,
 *    so a gate on qubit k pairs alpha_i with alpha_{i + 2^k} for i with bit k
 *    clear.  A bitstring x names the amplitude alpha_x, bit k = qubit k.
 *  - Arguments are validated on the host before anything is enqueued; a call
 *    that returns an error has enqueued nothing.  Errors never abort and
 *    never throw across the ABI.  qsv_last_error() returns a thread-local
 *    message for the last non-OK status of the calling thread.
 *  - Device faults surface as QSV_EHIP from the next call that synchronises.
 *  - Limits: n_qubits <= 34 for a single state (2^34 * 8 B = 128 GiB),
 *    bitstrings < 2^63, lattices up to 64 sites.  Device: gfx950 only.
 */
#ifndef QSV_PUBLIC_API_H_
#define QSV_PUBLIC_API_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QSV_OK = 0,
    QSV_EINVAL = 1,        /* bad argument: null pointer, bad kind, bad size */
    QSV_ERANGE = 2,        /* n too large, qubit or bitstring out of range */
    QSV_ENOMEM = 3,        /* host or device allocation failed */
    QSV_EHIP = 4,          /* HIP runtime error (message in qsv_last_error) */
    QSV_EUNSUPPORTED = 5,  /* option or device not supported (e.g. not gfx950) */
    QSV_EINTERNAL = 6
} qsv_status;

/*
 * Gate kinds.  The random circuit family uses H, T, SX = X^1/2, SY = Y^1/2
 * and CZ (Section 2, "universal random quantum circuit").  Matrices (rows
 * and columns indexed by the acted-on bit):
 *   H  = [[1,1],[1,-1]]/sqrt2            T   = diag(1, e^{i pi/4})
 *   SX = [[1+i,1-i],[1-i,1+i]]/2          SY  = [[1+i,-1-i],[1+i,1+i]]/2
 *   CZ = diag(1,1,1,-1) on (q0, q1)       Z   = diag(1,-1)
 *   P0 = |0><0|, P1 = |1><1| (projectors of the CZ split, Section 2)
 *   TDG, SXDG, SYDG = adjoints of T, SX, SY.
 * PB and ZB are the branch-parameterised gates that circuit_split emits for
 * a cut CZ: with l = bit `arg` of the branch index passed to sv_apply_*,
 * PB applies P_l and ZB applies Z^l.
 */
typedef enum {
    QSV_H = 0, QSV_T = 1, QSV_SX = 2, QSV_SY = 3, QSV_CZ = 4,
    QSV_P0 = 5, QSV_P1 = 6, QSV_Z = 7, QSV_TDG = 8, QSV_SXDG = 9, QSV_SYDG = 10,
    QSV_PB = 11, QSV_ZB = 12
} qsv_gate_kind;

/* One gate.  q1 is used by CZ only; arg is the branch bit of PB/ZB. */
typedef struct {
    uint8_t kind;
    uint8_t q0;
    uint8_t q1;
    uint8_t arg;
    uint16_t layer;   /* circuit layer, 0 = the opening Hadamard layer */
    uint16_t reserved;
} qsv_gate;

typedef struct qsv_circuit qsv_circuit;  /* opaque, host-owned */
typedef struct qsv_batch qsv_batch;      /* opaque */

/*
 * Tuning options of the fused sweep.  Pass NULL to let the autotuner pick.
 * A field left at 0 means "tuner's choice".
 *   reg_qubits     qubits held in each thread's registers (R, 3..6)
 *   thread_qubits  log2 of the workgroup size (T, 6..9); a tile holds
 *                  2^(R+T) amplitudes
 *   low_qubits     minimum number of always-resident low index bits that make
 *                  each global access a contiguous run (c, 3..8)
 *   plain          1 = one kernel per gate (the unfused comparator path)
 *   jit            1 = compile each pass program into its own straight-line
 *                  kernel at first use (hipRTC, cached per process), one tile
 *                  per workgroup; 2 = the same kernels as persistent workgroups
 *                  that prefetch their next tile into registers while they
 *                  compute the current one; 3 = per pass: pass p persistent iff
 *                  bit p of pass_forms is set (p < 19); 4 = as 1, but each
 *                  LDS exchange staged whole rather than in two halves (half
 *                  the buffer, twice the workgroups per CU, twice the
 *                  barriers: 1 stages in halves from 32 KiB buffers); -1 = always use the
 *                  generic pass kernel; 0 = 1 for states of 2^24 amplitudes or
 *                  more, else -1 (the environment variable QSV_JIT=0 makes 0
 *                  mean -1 everywhere; QSV_JIT_DUMP=<file> writes the last
 *                  generated source there, a debugging aid)
 *   out_of_place   compiled kernels only.  1 = every pass reads one buffer and
 *                  writes the other (the caller's state and the second state
 *                  buffer in the call's workspace, see sv_workspace_bytes), so
 *                  that each pass can write the state with the next pass's
 *                  qubits at the lowest address bits; the result is always in
 *                  the caller's buffer; QSV_EINVAL if the workspace cannot hold
 *                  the second buffer.  -1 = in place.  0 = out of place for
 *                  2^24 amplitudes or more when the workspace holds the second
 *                  buffer, else in place.
 *   pass_forms     see jit = 3.
 */
typedef struct {
    int reg_qubits;
    int thread_qubits;
    int low_qubits;
    int plain;
    int jit;
    int out_of_place;
    uint32_t pass_forms;
} qsv_fuse_opts;

/*
 * circuit_create - build a random lattice circuit or wrap an explicit list.
 *
 * Lattice: rows x cols sites; present[r*cols + c] != 0 marks a site that
 * holds a qubit (NULL = all present).  Qubit q is the row-major rank of its
 * site among the present ones.
 * Random circuit (gates == NULL): layer 0 is H on every qubit; layer
 * t = 1..depth applies the CZ pattern of class ORDER[(t-1) mod 8], then a
 * single-qubit gate drawn uniformly from {T, SX, SY} on every qubit that was
 * in a CZ at layer t-1 and is in none at layer t.  Pattern classes:
 *   Hab = horizontal bonds (r,c)-(r,c+1) with c = a, r = b (mod 2),
 *   Vab = vertical bonds (r,c)-(r+1,c) with r = a, c = b (mod 2),
 *   ORDER = H00, H01, V10, V11, H10, V01, V00, H11.
 * The gate types come from SplitMix64(seed), one draw per single-qubit gate
 * in gate order, type = floor((r >> 32) * 3 / 2^32) -> T, SX, SY.  These
 * rules are the reading that reproduces the gate counts of Table "28qubit"
 * and the cut counts of Section 2.1.2 (the paper defers them to the
 * random-circuit literature).
 * Explicit list (gates != NULL): the n_gates gates are copied; depth and seed
 * are ignored; every qubit index must be < the number of present sites.
 * On success *out owns a new circuit; free it with circuit_destroy.
 */
qsv_status circuit_create(int rows, int cols, const uint8_t *present, int depth,
                          uint64_t seed, const qsv_gate *gates, size_t n_gates,
                          qsv_circuit **out);
void circuit_destroy(qsv_circuit *c);
qsv_status circuit_info(const qsv_circuit *c, int *n_qubits, int *depth, size_t *n_gates);
/* Copy up to cap gates into out; *n_written = number copied. */
qsv_status circuit_gates(const qsv_circuit *c, qsv_gate *out, size_t cap, size_t *n_written);

/*
 * circuit_split - Schmidt split across a qubit bipartition (Section 2,
 * CU = P0 (x) I + P1 (x) U; Fig. 2).
 *
 * side_a_mask selects the side-A qubits (bit q = qubit q).  Every CZ with one
 * qubit on each side is either
 *   - folded: no non-diagonal gate follows on either qubit, so the CZ is the
 *     output phase (-1)^{x_a x_b} (e.g. the final layer), or
 *   - cut: it becomes branch bit j (j = 0,1,... in gate order): PB(j) on the
 *     side-A qubit and ZB(j) on the side-B qubit.
 * half_a / half_b receive new circuits over the side's qubits, renumbered in
 * increasing global order (local qubit i = i-th set bit of the side's mask).
 * *c_eff = number of cut CZs (2^c_eff branches).  The folded pairs are
 * written to folded_a[i], folded_b[i] (global qubit numbers, side A first)
 * for i < min(cap, count); *n_folded = count.  folded_a/folded_b may be NULL
 * when cap is 0.
 */
qsv_status circuit_split(const qsv_circuit *c, uint64_t side_a_mask,
                         qsv_circuit **half_a, qsv_circuit **half_b, int *c_eff,
                         int32_t *folded_a, int32_t *folded_b, size_t cap,
                         size_t *n_folded);

/*
 * circuit_inverse - the adjoint circuit U^dagger: gates in reverse order,
 * each replaced by its adjoint (T <-> TDG, SX <-> SXDG, SY <-> SYDG; H, CZ,
 * Z, ZB and the projectors P0, P1, PB are their own adjoints), layer numbers
 * mirrored (layer' = max layer - layer).  *out is a new host-owned circuit.
 */
qsv_status circuit_inverse(const qsv_circuit *c, qsv_circuit **out);

/*
 * Branch stages for prefix sharing among the branches of a split half (the
 * CZ decomposition of Section 2, Fig. 2: every branch runs the same gates
 * apart from the PB / ZB gates of its branch bits).
 *
 * The layers that hold PB / ZB gates, in ascending order, define levels
 * 1..L: level k fixes the branch bits of the k-th such layer.  Every gate
 * belongs to the deepest level among the branch bits it depends on through a
 * chain of gates that share a qubit and do not commute (two diagonal gates
 * commute), level 0 if it depends on none.
 *
 * circuit_branch_levels: *n_levels = L; level_bits[k] = mask of the branch
 * bits fixed at level k + 1, for k < min(L, cap) (level_bits may be NULL when
 * cap is 0).
 *
 * circuit_branch_stage: *out = new host-owned circuit (same n, depth and
 * layer numbers) with the gates of levels [level_begin, level_end) in their
 * original order; level_end = -1 means L + 1.  For any branch b and any
 * 0 = l0 < l1 < ... < lk = L + 1, running the stages [l0, l1), ...,
 * [l(k-1), lk) one after the other with branch b gives the same state as the
 * whole circuit with branch b (a gate only moves ahead of gates of a deeper
 * level, and only when the two commute).  A branch tree computes each stage
 * once per value of the branch bits of the levels before its end: the gates
 * of level 0 once, those of level 1 once per value of the level-1 bits, and
 * so on.  Errors: QSV_EINVAL for an empty range or one outside [0, L + 1).
 */
qsv_status circuit_branch_levels(const qsv_circuit *c, int *n_levels, uint64_t *level_bits, size_t cap);
qsv_status circuit_branch_stage(const qsv_circuit *c, int level_begin, int level_end, qsv_circuit **out);

/*
 * sv_init - write a basis or uniform state into amps (device complex64[2^n]).
 *   kind 0 = |0...0>, 1 = |+>^n (every amplitude 2^{-n/2}, i.e. layer 0
 *   applied), 2 = |basis>.  The simulated circuits start from |0...0> and
 *   open with a Hadamard on every qubit (Section 2, the random circuit
 *   rules); |basis> is the start of the adjoint half-sweep of Task 2
 *   (Section 2.2).  QSV_ERANGE for basis >= 2^n; asynchronous on stream.
 */
enum { QSV_INIT_ZERO = 0, QSV_INIT_PLUS = 1, QSV_INIT_BASIS = 2 };
qsv_status sv_init(void *amps, int n_qubits, int kind, uint64_t basis, void *stream);

/*
 * sv_workspace_bytes - size of the caller-owned workspace that the sweep
 * calls below (sv_apply_fused, sv_apply_fused_from, sv_simulate,
 * sv_simulate_dot, sv_simulate_c128, the sampler runs and sv_tune) use for
 * layers [layer_begin, layer_end) of c with these options (NULL = the tuned
 * or default ones).  It holds the second state buffer of out-of-place passes
 * (8 * 2^n bytes, when the options choose them) and the FP64 partial sums of
 * the norm and inner-product reductions (16 bytes per tile of the smallest
 * tile the tuner considers, at least 1 MiB), so a workspace sized before
 * sv_tune also fits the tuned shape.  Host only.  The library keeps no
 * pointer to a workspace past the call that receives it; two calls in flight
 * at once need two workspaces.
 */
qsv_status sv_workspace_bytes(const qsv_circuit *c, int layer_begin, int layer_end,
                              const qsv_fuse_opts *opts, size_t *bytes);

/*
 * sv_apply_fused - apply the gates of layers [layer_begin, layer_end) of the
 * circuit to amps in place (device complex64[2^n], n = the circuit's qubit
 * count).  layer_end < 0 means "to the end".  branch selects P_l / Z^l of the
 * PB/ZB gates (bit j of branch = l_j); ignored for circuits without them.
 *
 * The gates are grouped into full-state passes: each pass streams every
 * amplitude from HBM once, applies all gates it can on a tile of 2^(R+T)
 * amplitudes (non-diagonal gates on the tile's resident qubits, diagonal
 * T/CZ/Z/P gates on any qubit) and writes it back - the batching of gates on
 * "local" qubits and the free application of diagonal gates of Section 2.4.
 * Plans are built on the host on first use and cached in the circuit.
 * Asynchronous on stream; the state is exact (up to FP32 rounding) after the
 * last pass of the call, so calls over consecutive layer ranges compose.
 * workspace: caller-owned device memory of ws_bytes bytes (see
 * sv_workspace_bytes) or NULL; without room for the second state buffer the
 * passes run in place.  No device memory is allocated or freed by the call
 * (the first call of a plan compiles and loads its kernels).
 */
qsv_status sv_apply_fused(void *amps, const qsv_circuit *c, uint64_t branch,
                          int layer_begin, int layer_end, const qsv_fuse_opts *opts,
                          void *workspace, size_t ws_bytes, void *stream);

/*
 * sv_simulate - the whole sweep of one circuit in one call: initial state,
 * layers [layer_begin, layer_end), FP64 norm, gather.  Same result as
 * sv_init + sv_apply_fused + sv_norm_fp64 + sv_amplitudes, but on the
 * compiled-pass path the initial state (kind and basis as in sv_init) is
 * generated in registers by the first pass instead of being written and read
 * back, and the last pass accumulates the FP64 norm of the tiles it stores,
 * saving two full-state sweeps.  norm_out_dev (device double[1]) may be NULL;
 * with m = 0 nothing is gathered.  opts->plain selects the unfused path.
 * The init kinds are those of sv_init (Section 2: the opening Hadamard
 * layer makes |+>^n from |0>).  workspace / ws_bytes as for
 * sv_apply_fused; the norm needs it (its partial sums live there:
 * QSV_EINVAL without a workspace of sv_workspace_bytes bytes).  With m > 0
 * the bitstrings are range-checked as in sv_amplitudes, after the plan is
 * built and before anything is enqueued (the call then waits for the work
 * already queued on stream; QSV_ERANGE enqueues nothing).
 */
qsv_status sv_simulate(void *amps, const qsv_circuit *c, uint64_t branch, int init_kind,
                       uint64_t basis, int layer_begin, int layer_end, const qsv_fuse_opts *opts,
                       double *norm_out_dev, const uint64_t *bitstrings_dev, size_t m,
                       void *amps_out_dev, int out_c128, void *workspace, size_t ws_bytes,
                       void *stream);

/*
 * sv_simulate_dot - <U |init> | other> in FP64 without storing U |init>:
 * the sweep of sv_simulate (initial state generated by its first pass) whose
 * last pass reads `other` at the addresses it would write and accumulates
 * conj(result) * other, every product of the FP32 values exact in FP64,
 * summed in a fixed order (per tile, then over tiles).  With U = (layers
 * [h, end])^dagger (circuit_inverse), init = |x> and other = U1 |+> this is
 * the Task-2 amplitude <x| U2 U1 |+> of Section 2.2 in one call after the
 * forward half.  amps: work buffer for the passes before the last
 * (complex64[2^n], contents unspecified afterwards); other: device
 * complex64[2^n], not written; out_dev: device double[2] = (re, im).  With
 * the generic kernel the result is stored to amps and the inner product
 * follows.  workspace (required: the FP64 partial sums live there) and
 * ws_bytes as for sv_simulate.  Asynchronous on stream.
 */
qsv_status sv_simulate_dot(void *amps, const qsv_circuit *c, uint64_t branch, int init_kind,
                           uint64_t basis, int layer_begin, int layer_end, const qsv_fuse_opts *opts,
                           const void *other, double *out_dev, void *workspace, size_t ws_bytes,
                           void *stream);

/*
 * sv_simulate_c128 - the same sweep on a complex128 state (device
 * complex128[2^n], 16 bytes per amplitude): the compiled pass kernels
 * instantiated in FP64.  A precision reference for the complex64 path, not a
 * fast path; tile shape fixed at 4 register x 8 thread qubits, in place.
 * Output amplitudes are complex128[m]; norm_out_dev may be NULL (else the
 * norm's partial sums go to workspace, as for sv_simulate).  Needs
 * 12 <= n <= 34.  Bitstrings are range-checked as in sv_amplitudes.
 */
qsv_status sv_simulate_c128(void *amps, const qsv_circuit *c, uint64_t branch, int init_kind,
                            uint64_t basis, int layer_begin, int layer_end, double *norm_out_dev,
                            const uint64_t *bitstrings_dev, size_t m, void *amps_out_dev,
                            void *workspace, size_t ws_bytes, void *stream);

/*
 * sv_apply_fused_from - dst = U(layers [layer_begin, layer_end), branch) src
 * out of place: the same sweep as sv_apply_fused, with the first pass reading
 * src, which is never written (any pass count ends in dst).  For branch
 * trees of a cut circuit (Section 2, CU = P0 (x) I + P1 (x) U): branches
 * share every gate before their first differing cut, so the state at a cut
 * layer is computed once and each child continues from it.  src, dst:
 * device complex64[2^n], 16-byte aligned, must not overlap (src == dst runs
 * in place).  With the generic kernel (jit = -1) or the per-gate path, src
 * is copied to dst first.  workspace / ws_bytes as for sv_apply_fused.
 * Asynchronous on stream.
 */
qsv_status sv_apply_fused_from(const void *src, void *dst, const qsv_circuit *c, uint64_t branch,
                               int layer_begin, int layer_end, const qsv_fuse_opts *opts,
                               void *workspace, size_t ws_bytes, void *stream);

/*
 * sv_apply_plain - the unfused comparator: one full-state (or, for diagonal
 * gates, partial) kernel per gate, the gate-by-gate method that Section 2.4
 * and Table "28qubit" measure their speedup against.  Same arguments and
 * result as sv_apply_fused.
 */
qsv_status sv_apply_plain(void *amps, const qsv_circuit *c, uint64_t branch,
                          int layer_begin, int layer_end, void *stream);

/*
 * sv_apply_dense - apply layers [layer_begin, layer_end) as dense blocks on
 * matrix cores.  The gates are grouped into blocks that each act on k qubits
 * (k = 4, 5 or 6); every block's 2^k x 2^k complex matrix is formed in FP64
 * on the host (product of its gate matrices, rounded to complex64) and
 * applied to the state in one full pass with FP32 MFMA (Y = M X, X = the
 * columns of 2^k amplitudes that share all other index bits).  This is gate
 * fusion in the sense of the qHiPSTER comparison of Section 2.4: cost
 * 8 * 2^k real flops per amplitude per block.  *n_blocks (may be NULL)
 * receives the number of blocks.  Requires n >= k + 6.
 */
qsv_status sv_apply_dense(void *amps, const qsv_circuit *c, uint64_t branch, int layer_begin,
                          int layer_end, int k, int *n_blocks, void *stream);

/*
 * Sampling from a parent state: amplitudes of U src at a fixed set of m
 * bitstrings, where U = the gates of layers [layer_begin, layer_end) with
 * the branch bits of each run.  For the leaves of a branch tree (Task 2 over
 * cut circuits, Section 2.2 / Fig. 2) only sampled amplitudes of each leaf
 * are needed: the last pass of the sweep runs only the tiles that hold a
 * requested index (at most m of them) and writes those amplitudes instead
 * of the state, so the leaf's state is never stored.
 * sv_sampler_create: plans the sweep, groups the bitstrings (host array,
 *   each < 2^n, copied) by the last pass's tile and prepares the kernels;
 *   the circuit must stay alive until sv_sampler_destroy.
 * sv_sampler_run: out_dev[k] (device complex64[m]) = (U src)[bitstrings[k]];
 *   src: device complex64[2^n], not written; work: another device
 *   complex64[2^n] for the passes before the last (contents unspecified
 *   afterwards).  With the generic kernel the sweep is stored to work and
 *   gathered.  The sampler's plan is fixed when it is created: when it runs
 *   out of place (the options choose it, see sv_workspace_bytes) every run
 *   needs a workspace that holds the second state buffer (QSV_EINVAL
 *   otherwise).  Asynchronous on stream.
 * sv_sampler_run_branches: sv_sampler_run for count branches of the same
 *   src, one after the other on the stream (the sibling leaves of a branch
 *   tree): branches = host uint64[count], out_dev = device
 *   complex64[count * m], row i for branches[i].  Stops at the first error.
 * sv_sampler_run_subtree: the 2^k sibling branches prefix | (bits of y
 *   deposited on the k set bits of mask), y = 0 .. 2^k - 1, from the same
 *   src: row y of out_dev (device complex64[2^k * m]) for the y-th.  When the
 *   sweep is one compiled pass this is one launch whose grid holds a row of
 *   workgroups per branch (the leaves of a branch tree at once); otherwise
 *   one run per branch.  prefix & mask must be 0 (QSV_EINVAL); k <= 15
 *   (QSV_ERANGE).
 * sv_sampler_create_tiles: a sampler whose last pass computes the tiles that
 *   hold the given indices and stores each of them whole: sv_sampler_run
 *   then writes (U src) at every index of those tiles (a superset of the
 *   given ones) into out_dev, a device complex64[2^n] that is neither src nor
 *   work, and leaves the rest of out_dev untouched.  For the inner levels of
 *   a branch tree whose leaves read only part of their parent.  Needs the
 *   compiled pass kernels (QSV_EUNSUPPORTED otherwise); run_branches and
 *   run_subtree refuse it (QSV_EINVAL).
 * sv_sampler_inputs: for a sampler whose sweep is one compiled pass, the
 *   indices of src its run reads (the amplitudes of the tiles it computes):
 *   *count = their number, the first min(cap, *count) written to out (host
 *   uint64).  QSV_EUNSUPPORTED when the run reads the whole state.
 */
typedef struct qsv_sampler qsv_sampler;  /* opaque */
qsv_status sv_sampler_create(const qsv_circuit *c, int layer_begin, int layer_end, const qsv_fuse_opts *opts,
                             const uint64_t *bitstrings, size_t m, qsv_sampler **out);
qsv_status sv_sampler_run(qsv_sampler *s, const void *src, void *work, uint64_t branch, void *out_dev,
                          void *workspace, size_t ws_bytes, void *stream);
qsv_status sv_sampler_run_branches(qsv_sampler *s, const void *src, void *work, const uint64_t *branches,
                                   size_t count, void *out_dev, void *workspace, size_t ws_bytes,
                                   void *stream);
qsv_status sv_sampler_run_subtree(qsv_sampler *s, const void *src, void *work, uint64_t prefix, uint64_t mask,
                                  void *out_dev, void *workspace, size_t ws_bytes, void *stream);
qsv_status sv_sampler_create_tiles(const qsv_circuit *c, int layer_begin, int layer_end,
                                   const qsv_fuse_opts *opts, const uint64_t *indices, size_t m,
                                   qsv_sampler **out);
qsv_status sv_sampler_inputs(const qsv_sampler *s, uint64_t *out, size_t cap, size_t *count);
void sv_sampler_destroy(qsv_sampler *s);

/*
 * sv_amplitudes - gather alpha_x for m bitstrings (Task 2 of Section 1).
 * bitstrings_dev: device uint64[m]; out_dev: device complex64[m]
 * (out_c128 = 0) or complex128[m] (out_c128 = 1).  Range check: before
 * anything is enqueued, a small kernel tests every bitstring against 2^n and
 * the call waits for the stream (so for the work queued before it); a
 * bitstring >= 2^n returns QSV_ERANGE with nothing enqueued.  On a stream
 * under graph capture the wait is impossible: the check is skipped and the
 * gather writes NaN for such entries.  Otherwise asynchronous on stream.
 */
qsv_status sv_amplitudes(const void *amps, int n_qubits, const uint64_t *bitstrings_dev,
                         size_t m, void *out_dev, int out_c128, void *stream);

/*
 * sv_stream_copy - dst = src for `bytes` bytes of device memory (a multiple
 * of 16; both buffers 16-byte aligned and disjoint) with the access pattern
 * of the fused passes: 16-byte nontemporal loads and stores, several in
 * flight per thread.  The HBM rate of a pass without arithmetic, the
 * ceiling the sweep's rate is compared with (one read and one write per
 * amplitude, like one pass).  Asynchronous on stream.
 */
qsv_status sv_stream_copy(const void *src, void *dst, size_t bytes, void *stream);

/*
 * sv_norm_fp64 - sum of |alpha_i|^2 over the state with every product and
 * partial sum in FP64 and a fixed-order pairwise tree (deterministic): the
 * norm check of the sweep (a unitary circuit keeps it at 1).  out_dev:
 * device double[1].  The partial sums go to a 1 MiB buffer that the library
 * allocates for each device and stream on its first such call (freed by
 * qsv_release_device_buffers); calls on different streams never share one.
 */
qsv_status sv_norm_fp64(const void *amps, int n_qubits, double *out_dev, void *stream);

/*
 * sv_norm_fp64_noalloc - sv_norm_fp64 for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops and
 * harnesses that forbid hipMalloc.  Same kernels, same result bit for bit;
 * the partial sums live in a fixed device array of 65536 doubles (512 KiB)
 * that each GPU holds from the first call on it until the process ends.
 * The call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine).  Calls that overlap on one device share that array and race:
 * serialise them (one stream, or events between streams).  n_qubits <= 34
 * (QSV_ERANGE otherwise); the state needs at most 65536 partials at any n.
 */
qsv_status sv_norm_fp64_noalloc(const void *amps, int n_qubits, double *out_dev, void *stream);

/*
 * sv_inner_product - <a|b> = sum_i conj(a_i) b_i of two complex64[2^n]
 * device states, every product and partial sum in FP64, fixed-order tree
 * (deterministic).  out_dev: device double[2] = (re, im).  With a = U2^dagger
 * |x> and b = U1 |psi0> this is the Task-2 amplitude <x|U2 U1|psi0> of
 * Section 2.2 from two half-depth sweeps.
 */
qsv_status sv_inner_product(const void *a, const void *b, int n_qubits, double *out_dev,
                            void *stream);

/*
 * sv_branch_combine - out[x] = s_x * sum_b a_tab[b][x] * b_tab[b][x]
 * (Fig. 2 and eq. (1): the output is the sum over branches of the tensor
 * product of the two half states, here at m sampled bitstrings).
 * a_tab, b_tab: device complex64[n_branches][m] (branch-major); sign_dev:
 * device int8[m] of +1/-1 (the folded phases) or NULL for all +1; out_dev:
 * device complex128[m].  Products and sums in FP64, fixed pairwise order.
 */
qsv_status sv_branch_combine(const void *a_tab, const void *b_tab, size_t n_branches,
                             size_t m, const int8_t *sign_dev, void *out_dev, void *stream);

/*
 * sv_branch_combine_full - the complete state of a cut circuit (Fig. 2,
 * eq. (1), eqs. (6)-(7)): out[x] = s(x) * sum_b A_b[x_A] B_b[x_B] for all
 * 2^(n_a + n_b) indices x, a complex GEMM on matrix cores.  flags = 0: the
 * complex64 inputs are widened to FP64 and every product and sum is FP64
 * (v_mfma_f64_16x16x4f64), the result rounded once to a complex64 out_state;
 * QSV_COMBINE_OUT_C128: out_state is complex128 (no rounding);
 * QSV_COMBINE_FP32: FP32 products and accumulation on FP32 matrix cores
 * (twice the rate, FP32 rounding in the sums).  a_states: complex64
 * [n_branches][2^n_a] (branch-major),
 * local qubit i of side A = i-th set bit of side_a_mask; b_states likewise
 * for the other n_b qubits (as circuit_split numbers them).  folded_a /
 * folded_b: the folded pairs of circuit_split (global qubit numbers, side A
 * first), s(x) = (-1)^{sum x_a x_b}.  out_state: complex64[2^(n_a+n_b)] in
 * natural order.  Limits: 7 <= n_a, 7 <= n_b <= 22, n_a + n_b <= 34, at most
 * 64 folded pairs.  All buffers are caller-owned device memory.
 */
enum { QSV_COMBINE_OUT_C128 = 1, QSV_COMBINE_FP32 = 2 };
qsv_status sv_branch_combine_full(const void *a_states, const void *b_states, size_t n_branches,
                                  int n_a, int n_b, uint64_t side_a_mask, const int32_t *folded_a,
                                  const int32_t *folded_b, size_t n_folded, void *out_state, int flags,
                                  void *stream);

/*
 * Batched execution: many states (branches of split halves, or independent
 * circuits of uneven size) swept together, replayed from a captured hipGraph
 * (Section 3: Stage 1 runs many independent sub-circuit sweeps; Fig. 2: the
 * branches of a cut circuit).
 *
 * Size classes.  States of at most 2^14 amplitudes run on a tile that holds
 * the whole state (the whole circuit in one workgroup, in registers and LDS);
 * states below 2^21 amplitudes on the batch's tile shape; both with the
 * generic pass kernel, one launch per tile shape and pass round.  States of
 * 2^21 amplitudes or more run compiled kernels of their own plan on the tile
 * shape tuned for their class (sv_tune / sv_tune_set); in the captured graph
 * each such plan's chain of passes is a branch of its own, so independent
 * states run side by side (the batch makes four side streams for the
 * capture when it has two or more such plans).  A persistent form
 * (one launch per tile shape whose workgroups take work items (pass round,
 * entry, tile) in order from a device counter, per-entry counters of
 * completed tiles ordering each entry's passes) is switched off in this
 * version: QSV_BATCH_PERSISTENT=1 makes sv_batch_create return
 * QSV_EUNSUPPORTED.
 *
 * sv_batch_create: count entries; entry i runs circuit circs[i] with branch
 * index branch_ids[i] (NULL = all 0) on its own state.  Plans per circuit
 * are built here.  opts may force one tile shape for every generic entry
 * ((5,9), (5,8), (5,7), (4,8) or (4,7)) and the compiled-kernel mode (jit).
 * The circuits must stay alive until sv_batch_destroy.  States need >= 11
 * qubits.
 * sv_batch_run: amps_dev[i] is entry i's device state (complex64[2^n_i]),
 * already initialised by the caller (or pass init_plus = 1 to have the
 * launch start every state from |+>^n itself).  After the sweep, when
 * m > 0, the amplitudes at bitstrings_dev[i*m .. i*m+m-1] (device uint64,
 * local numbering of entry i) are written to amp_table_dev[i*m + k] (device
 * complex64).  The first call captures a graph for these pointers; later
 * calls with the same pointers replay it.  Asynchronous on stream; the
 * bitstrings are not range-checked (the replayed graph cannot wait for a
 * check): an entry's bitstring >= 2^n_i gives NaN in its table slot.
 * sv_batch_status: synchronises stream and reports QSV_EINTERNAL if a wait of
 * a persistent launch gave up since the last status call (its bounded spin
 * ran out, or sv_batch_abort was called): the results of that run are then
 * unspecified.  Clears the abort request.
 * sv_batch_abort: asks the waits of the batch's launches in flight to give up
 * (host only; a pinned flag they poll), so every launch drains promptly.
 */
qsv_status sv_batch_create(const qsv_circuit *const *circs, const uint64_t *branch_ids,
                           size_t count, const qsv_fuse_opts *opts, qsv_batch **out);
qsv_status sv_batch_run(qsv_batch *b, void *const *amps_dev, int init_plus,
                        const uint64_t *bitstrings_dev, size_t m, void *amp_table_dev,
                        void *stream);
qsv_status sv_batch_status(qsv_batch *b, void *stream);
qsv_status sv_batch_abort(qsv_batch *b);
void sv_batch_destroy(qsv_batch *b);

/*
 * sv_tune - autotune the fused sweep of layers [layer_begin, layer_end) of c.
 * Candidate tile shapes (register qubits, thread qubits, always-resident low
 * qubits) are planned; those within one pass of the fewest passes are timed
 * on the device on amps_scratch (device complex64[2^n], contents destroyed)
 * with the workspace given (out-of-place forms are considered only when it
 * holds a second state buffer; see sv_workspace_bytes), the three fastest
 * also in the persistent form (jit = 2) and with exchanges staged whole
 * (jit = 4), and the fastest with each pass in the faster of forms 1 and 2
 * (jit = 3); the fastest of all is written to *out (and its median time in
 * ms to *best_ms, may be NULL).
 * States above 2^31 amplitudes are timed on the first 2^31 amplitudes' worth
 * of tiles of every pass; every timing is the median of five.  The choice is remembered for this circuit content
 * and layer range: later calls with opts == NULL use it.  This is the
 * scheduling preprocessing of Section 2.4 done by measurement.  Synchronises
 * the stream.  With the environment variable QSV_TUNE_CACHE=<file> the
 * choice is also appended to that file (keyed by a hash of the qubit count,
 * layer range, gate list and device) and a later process takes it from
 * there without timing; QSV_JIT_CACHE=<directory> likewise keeps the
 * compiled pass kernels' code objects (keyed by a hash of their source and
 * compiler options) so a later process loads them instead of compiling.
 */
qsv_status sv_tune(void *amps_scratch, const qsv_circuit *c, int layer_begin, int layer_end,
                   void *workspace, size_t ws_bytes, qsv_fuse_opts *out, double *best_ms,
                   void *stream);
/*
 * sv_tune_set - remember opts as the tuned options of c and the layer range,
 * as if sv_tune had picked them (host only).  A batch tunes one circuit per
 * size class with sv_tune and hands the choice to the others of the class;
 * sv_batch_create gives states of 2^21 amplitudes or more the tile shape
 * tuned for their circuit (the default shape otherwise).
 */
qsv_status sv_tune_set(const qsv_circuit *c, int layer_begin, int layer_end, const qsv_fuse_opts *opts);

/*
 * Plan inspection (host only, no device needed).  For the plan that
 * sv_apply_fused would use: *n_passes, and for each gate of the layer range
 * the pass it runs in (pass_of_gate[i], -1 if outside the range) and its
 * position in that pass's program (order_in_pass[i]); resident_mask[p] is
 * the bit set of qubits resident in pass p (cap entries).  Arrays may be
 * NULL.  Used by tests to check the grouping against the gate semantics.
 */
qsv_status sv_plan_info(const qsv_circuit *c, int layer_begin, int layer_end,
                        const qsv_fuse_opts *opts, int *n_passes, int32_t *pass_of_gate,
                        int32_t *order_in_pass, size_t n_gate_cap, uint64_t *resident_mask,
                        size_t pass_cap);

/*
 * sv_debug_emulate - run the fused plan's pass programs on the host over a
 * host complex64[2^n] array, with the same slot/exchange semantics as the
 * GPU kernel.  A planner/encoding check for CPU-only test runs; never used
 * by sv_apply_fused or any other entry point.
 */
qsv_status sv_debug_emulate(void *amps_host, const qsv_circuit *c, uint64_t branch,
                            int layer_begin, int layer_end, const qsv_fuse_opts *opts);

/*
 * sv_debug_batch_schedule - host emulation of the work-item schedule of a
 * persistent batch launch (a CPU check of its ordering rule; no product entry
 * point calls it): count entries of n_qubits[i] qubits and passes[i] passes on
 * tiles of 2^tile_qubits amplitudes, `workers` virtual workgroups taking the
 * items in order, completions in a seeded random order.  QSV_OK if every
 * (entry, pass, tile) runs exactly once, none starts before every tile of its
 * entry's earlier passes has completed, and nothing stalls; QSV_EINTERNAL
 * otherwise.  *items_out (may be NULL) = the launch's work items.
 * planted_early_start != 0 lets an item start one completed tile early (a
 * planted mistake that the check must catch).
 */
qsv_status sv_debug_batch_schedule(const int *n_qubits, const int *passes, size_t count, int tile_qubits,
                                   int workers, uint64_t seed, int planted_early_start, uint64_t *items_out);

/*
 * sv_debug_emulate_dense - apply the dense blocks of sv_apply_dense on the
 * host to a complex64[2^n] host array (n <= 24).  A block-construction check
 * for CPU-only test runs; no product entry point calls it.
 */
qsv_status sv_debug_emulate_dense(void *amps_host, const qsv_circuit *c, uint64_t branch,
                                  int layer_begin, int layer_end, int k, int *n_blocks);

/*
 * sv_debug_jit_compile - generate and compile (no load, no device needed) the
 * straight-line kernels of the plan sv_apply_fused would use; reports the
 * code-object size and compile time.  A code-generation check for CPU-only
 * test runs.
 */
qsv_status sv_debug_jit_compile(const qsv_circuit *c, int layer_begin, int layer_end,
                                const qsv_fuse_opts *opts, size_t *code_bytes, double *seconds);

/*
 * Three-part partition (Section 2.1.1: implicit decomposition, eqs. (2)-(3);
 * Section 2.1.2: the dynamic programme of Algorithm 1).
 *
 * The circuit must be a lattice circuit (rows x cols, present mask as for
 * circuit_create, qubit = row-major rank among present sites) without branch
 * gates.  Two splitting lines run between lattice rows.  Initially both lie
 * between rows r0-1 and r0: part A's qubits are the sites with row < r0,
 * part B's the others.  From the separation layer t_s (1..depth+1) on, the
 * upper line sits ups[k] rows higher and the lower line dns[k] rows lower in
 * column k (non-decreasing over layers); at a layer t >= t_s a site (r, k)
 * belongs to A if r < r0 - ups[k], to B if r >= r0 + dns[k], else to part C.
 * Every CZ of layers 1..t_s-1 joining the two sides is cut (CZ = sum_l Z^l
 * (x) P_l); from t_s on no CZ may join two different parts.  Then
 * psi_out = U_C sum_l phi_l (x) xi_l: the gates of part C act on the block of
 * each fixed value of the other qubits independently.
 *
 * A cut is free on a side when its qubit there receives no non-diagonal gate
 * of that part after the cut: the projector is then absorbed (that side needs
 * no branch bit; the other side's branch is selected by the qubit's value).
 * A cut free on both sides is the output sign (-1)^{x_a x_b}.  Space exponents
 * f = n_A + (cuts not free on A), g = n_B + (cuts not free on B), n_c = size
 * of part C after the last layer.
 *
 * circuit_partition_plan: Algorithm 1 for both lines (offsets capped by
 *   max_move and the rows available) for every separation layer; keeps the
 *   scheme with the smallest 2^f + 2^g + 2^n_c.
 * circuit_partition_create: an explicit scheme; ups / dns hold
 *   (depth + 1 - t_s) x cols offsets (layer-major); QSV_EINVAL if illegal.
 * circuit_partition_offsets: the scheme's offsets (cap >= (depth+1-t_s)*cols).
 * circuit_partition_parts: copies of the three part circuits (caller
 *   destroys them).  A and B use local qubit numbers (qubits_a / qubits_b,
 *   may be NULL, receive the global qubit of each local one, n_a / n_b
 *   entries); their branch index holds the shared bits first, then the
 *   selector bits.  C uses global numbers.
 * All of these are host-only.
 */
typedef struct qsv_partition qsv_partition;  /* opaque, host-owned */
typedef struct {
    int r0, t_s, depth, cols;
    int n_a, n_b, n_c;       /* qubits of parts A, B and (after the last layer) C */
    int cuts;                /* cut CZ gates */
    int explicit_bits;       /* cuts with a branch bit on both sides */
    int sel_a, sel_b;        /* A (B) qubits whose value selects B's (A's) branch */
    int folded;              /* cuts folded into the output sign */
    int f, g;                /* space exponents of parts A and B */
    double objective;        /* 2^f + 2^g + 2^n_c */
    uint64_t branches_a;     /* branch states of part A: 2^(explicit_bits + sel_b) */
    uint64_t branches_b;     /* branch states of part B: 2^(explicit_bits + sel_a) */
} qsv_partition_info;

qsv_status circuit_partition_plan(const qsv_circuit *c, int rows, int cols, const uint8_t *present,
                                  int r0, int max_move, qsv_partition **out);
qsv_status circuit_partition_create(const qsv_circuit *c, int rows, int cols, const uint8_t *present,
                                    int r0, int t_s, const uint8_t *ups, const uint8_t *dns,
                                    qsv_partition **out);
qsv_status circuit_partition_info(const qsv_partition *p, qsv_partition_info *out);
qsv_status circuit_partition_offsets(const qsv_partition *p, uint8_t *ups, uint8_t *dns, size_t cap);
qsv_status circuit_partition_parts(const qsv_partition *p, qsv_circuit **a, qsv_circuit **b,
                                   qsv_circuit **c, int32_t *qubits_a, int32_t *qubits_b);
void circuit_partition_destroy(qsv_partition *p);

/*
 * sv_partition_simulate - psi_out of the circuit through its partition
 * (eqs. (2)-(3)) into out_state (device complex64[2^n], natural order):
 *   1. every branch state of parts A and B, from |+> with layer 0 folded in,
 *      into workspace: one batch (sv_batch_*) for the parts of 11 or more
 *      qubits, one sv_simulate call per branch for a smaller part;
 *   2. psi_in = s(x) sum_e phi_{e,u(x)}[x_A] xi_{e,w(x)}[x_B] (e = shared
 *      branch bits, u / w = the selector qubits' values) as complex GEMMs
 *      with FP64 products and sums on matrix cores, one per value of the
 *      selector qubits, rounded once to complex64;
 *   3. the gates of part C with sv_apply_fused on out_state.
 * workspace: device memory of sv_partition_workspace_bytes bytes (A's branch
 * states, then B's), caller-owned; the partition keeps the batch it built for
 * this workspace until it is destroyed, so the workspace must stay alive as
 * long as the partition is used with it.  Limits: n <= 34, n_a - sel_a >= 7,
 * 7 <= n_b - sel_b <= 22 (QSV_EUNSUPPORTED otherwise).  Asynchronous on
 * stream (the first call per workspace builds and captures the batch).
 * Calls on one partition must not overlap (they share its batch); part C
 * runs out of place in the library's second state buffer for n >= 24.
 */
qsv_status sv_partition_workspace_bytes(const qsv_partition *p, size_t *bytes);
qsv_status sv_partition_simulate(qsv_partition *p, void *workspace, size_t ws_bytes, void *out_state,
                                 void *stream);

/*
 * qsv_release_device_buffers - free the device memory the library keeps on
 * the current device between calls: the FP64 partial-sum buffers of
 * sv_norm_fp64 and sv_inner_product (1 MiB per stream that called them).
 * Synchronises the device first.  Later calls allocate again as needed.
 */
qsv_status qsv_release_device_buffers(void);

const char *qsv_last_error(void);
/* Library version string. */
const char *qsv_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QSV_PUBLIC_API_H_ */
