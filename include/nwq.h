/*
 * nwq.h -- C ABI of the MI355X (gfx950) state-vector / density-matrix engine.
 *
 * The engine implements the two simulators the paper's Sec. II describes
 * (a state-vector simulator for ideal circuits and a density-matrix simulator
 * for noise-aware runs), the noise model of Sec. III (depolarisation and
 * thermal relaxation, the latter as amplitude + phase damping), and the
 * observables of Sec. III (magnetisations <Z_i>, Pauli-sum energies, VQE
 * energies and gradients).  Choosing nwq_sv_create or nwq_dm_create plays
 * the role of choosing the simulator backend (Sec. II, Fig. 2).
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 *  - Qubit q is bit q of the basis index (little endian).  A k-qubit matrix
 *    on qubits (q_0, ..., q_{k-1}) is 2^k x 2^k, complex, row-major, with
 *    row/column index u = sum_j bit(q_j) 2^j.
 *  - Complex numbers are interleaved (re, im) FP64 pairs, i.e. the
 *    torch.complex128 / std::complex<double> layout.
 *  - SV state: 2^n complex amplitudes.  DM state: 4^n complex entries, the
 *    row-major vec of rho: entry (r, c) at index r * 2^n + c.
 *  - Pauli strings are (xmask, zmask) pairs: on qubit q, (x_q, z_q) =
 *    (0,0) I, (1,0) X, (1,1) Y, (0,1) Z.
 *  - Every function returns NWQ_OK (0) or a negative nwq_status.  On error
 *    the state is left unchanged (arguments are validated before any launch)
 *    and nwq_last_error() holds a message (thread-local).
 *  - Host arrays passed in are read during the call only; the caller keeps
 *    ownership.  Device pointers are never freed by the library unless the
 *    library allocated them.
 *  - apply_* calls are asynchronous on the handle's HIP stream.  Calls that
 *    return numbers to the host (expval, trace, purity, get_state)
 *    synchronise that stream.  A handle is not thread-safe; use one stream
 *    per handle.
 */
#ifndef NWQ_H
#define NWQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nwq_state* nwq_handle;

enum nwq_status {
  NWQ_OK = 0,
  NWQ_EINVAL = -1,    /* bad gate type, parameter count, size or pointer     */
  NWQ_ERANGE = -2,    /* qubit index >= n, or n outside the supported range  */
  NWQ_EDUP = -3,      /* the same qubit given twice                          */
  NWQ_EKIND = -4,     /* operation not valid on this handle kind (SV vs DM)  */
  NWQ_ENOTCPTP = -5,  /* Kraus set violates sum_k K^dag K = I beyond 1e-12   */
  NWQ_ENOMEM = -6,    /* device allocation failed                            */
  NWQ_EDEVICE = -7    /* a HIP runtime call failed (message kept)            */
};

/* Gate types (Sec. II circuits; Sec. III TFIM and VQE circuits).
 * Rotations are exp(-i theta P / 2); U3 follows OpenQASM 2:
 *   U3(t,p,l) = [[cos t/2, -e^{il} sin t/2], [e^{ip} sin t/2, e^{i(p+l)} cos t/2]].
 * Two-qubit gates list the control first (CX, CZ); RZZ = exp(-i t Z Z / 2). */
enum nwq_gate {
  NWQ_GATE_I = 0, NWQ_GATE_X, NWQ_GATE_Y, NWQ_GATE_Z, NWQ_GATE_H,
  NWQ_GATE_S, NWQ_GATE_SDG, NWQ_GATE_T, NWQ_GATE_TDG,
  NWQ_GATE_RX, NWQ_GATE_RY, NWQ_GATE_RZ, NWQ_GATE_U3,
  NWQ_GATE_CX, NWQ_GATE_CZ, NWQ_GATE_SWAP, NWQ_GATE_RZZ,
  NWQ_GATE_COUNT
};

enum nwq_kind { NWQ_KIND_SV = 0, NWQ_KIND_DM = 1 };

/* ---------------------------------------------------------------------------
 * Handles (Sec. II: the SV and DM simulators)
 * ------------------------------------------------------------------------- */

/* Create an SV state of n qubits (1 <= n <= 34) on `hip_stream` (a
 * hipStream_t, NULL = default stream); the library allocates 16 * 2^n bytes
 * of device memory and initialises |0...0>.  NWQ_ENOMEM if it does not fit. */
int nwq_sv_create(int n, void* hip_stream, nwq_handle* out);

/* Create a DM state of n qubits (1 <= n <= 17): 16 * 4^n bytes, rho = |0><0|. */
int nwq_dm_create(int n, void* hip_stream, nwq_handle* out);

/* Wrap caller-owned device memory (e.g. a torch complex128 tensor) of
 * 2^n (SV) or 4^n (DM) complex entries, 16-byte aligned.  The contents are
 * taken as the current state (no reset).  The library never frees it. */
int nwq_sv_create_from(void* dev_ptr, int n, void* hip_stream, nwq_handle* out);
int nwq_dm_create_from(void* dev_ptr, int n, void* hip_stream, nwq_handle* out);

/* Synchronise the stream and release everything the library allocated. */
int nwq_destroy(nwq_handle h);

/* Kind (nwq_kind), qubit count and device pointer of a handle. */
int nwq_info(nwq_handle h, int* kind, int* n, void** dev_ptr);

/* ---------------------------------------------------------------------------
 * State operations
 * ------------------------------------------------------------------------- */

/* Reset to |0...0> (SV) or |0...0><0...0| (DM), the initial state of the
 * Sec. III experiments, with a fill kernel (no memset node). */
int nwq_reset(nwq_handle h);

/* Copy the state to / from host memory of n_doubles = 2 * 2^n (SV) or
 * 2 * 4^n (DM) doubles (interleaved re, im).  get_state synchronises. */
int nwq_get_state(nwq_handle h, double* host, size_t n_doubles);
int nwq_set_state(nwq_handle h, const double* host, size_t n_doubles);

/* Launch any deferred work (fused DM superoperator, queued SV gates). */
int nwq_flush(nwq_handle h);

/* ---------------------------------------------------------------------------
 * Gates (Sec. II; SV: psi <- U psi, DM: rho <- U rho U^dag)
 * ------------------------------------------------------------------------- */

/* Apply gate `type` to `qubits` (n_q = 1 or 2, distinct, < n) with n_p
 * parameters (RX/RY/RZ/RZZ: 1, U3: 3, others: 0).  On a DM handle the
 * gate's superoperator U (x) conj(U) is held back so that the channels that
 * follow on the same qubits fuse into the same single pass over rho. */
int nwq_apply_gate(nwq_handle h, int type, const int* qubits, int n_q,
                   const double* params, int n_p);

/* Apply an arbitrary k-qubit matrix (k = 1 or 2; 2^k x 2^k complex,
 * row-major, interleaved) to `qubits`.  Unitarity is not checked on SV; on
 * DM it is applied as rho <- M rho M^dag. */
int nwq_apply_matrix(nwq_handle h, const int* qubits, int k, const double* m);

/* Apply the gates of a whole circuit: n_gates entries of types[],
 * qubits[2*i .. 2*i+1] (second entry ignored for 1-qubit gates) and
 * params[3*i .. 3*i+2] (unused entries ignored).  With fusion enabled on an
 * SV handle (nwq_set_fusion) consecutive gates are grouped into k-qubit
 * blocks, each applied in one pass through LDS. */
int nwq_apply_circuit(nwq_handle h, int n_gates, const int* types,
                      const int* qubits, const double* params);
/* Reset to |0...0> and apply the circuit (arguments as nwq_apply_circuit,
 * all validated before the reset).  With fusion on an SV handle, the first
 * block runs only on the tile that holds index 0: every other tile is zero
 * and a block maps each tile to itself, so they stay zero (the result equals
 * nwq_reset + nwq_apply_circuit, up to the sign of zero entries). */
int nwq_run_circuit(nwq_handle h, int n_gates, const int* types,
                    const int* qubits, const double* params);

/* OpenQASM 2.0 front-end (host only).  Accepts the header, include lines,
 * qreg / creg (quantum registers laid out in declaration order), the qelib1
 * gates id x y z h s sdg t tdg rx ry rz u1 u2 u3 u p cx CX cz swap rzz and
 * the built-in U with register broadcast, parameter expressions (numbers,
 * pi, + - * / ^, unary minus, parentheses, sin cos tan exp ln sqrt), and
 * skips barrier and measure.  u1(l) = p(l) = U3(0, 0, l); u2(f, l) =
 * U3(pi/2, f, l); rotations keep this library's exp(-i theta P / 2)
 * convention (equal to the textual qelib1 definitions up to a global
 * phase).  Gate definitions, if, reset and opaque give NWQ_EINVAL; every
 * error message names the line.
 *
 * nwq_qasm_parse writes the number of qubits and gates, and the first
 * min(capacity, gates) gates in the arrays of nwq_apply_circuit (call with
 * capacity 0 to size them).  nwq_apply_qasm parses and applies the program
 * (NWQ_ERANGE if its qubit count differs from the handle's); with fusion
 * enabled the whole program goes through the block planner. */
int nwq_qasm_parse(const char* text, int* n_qubits, int* n_gates, int capacity, int* types, int* qubits,
                   double* params);
int nwq_apply_qasm(nwq_handle h, const char* text);

/* Fused-block width: 0 = off (one kernel per gate), else the number of bits
 * a block may touch (6..13).  SV handles: nwq_apply_circuit runs its gates
 * through fused blocks.  DM handles: each 1q gate with the channels composed
 * after it (a 4x4 superoperator on bits q and q + n of vec(rho)) is queued,
 * and so is each 2q gate with its channels (a 16x16 on bits q0, q1, q0 + n,
 * q1 + n) when the fused kernel is 1 (4 register bits), n >= 4 and a block
 * can hold its four bits (2n <= k, or k minus the low tile bits of
 * nwq_set_fusion_lowbits is at least 4); the queue
 * runs as fused blocks over the 2n bits when a read or nwq_flush needs the
 * state, or a 2q superoperator that cannot be queued comes (a reset or
 * nwq_set_state drops it); changing the width or the fused kernel on a DM
 * handle flushes first.  Returns the value in effect through *k_out when
 * non-NULL. */
int nwq_set_fusion(nwq_handle h, int k, int* k_out);

/* Low tile bits of fused blocks: every block's tile holds the lowest c bits
 * of the index (contiguous runs of 2^c entries in HBM) plus up to k - c high
 * bits its gates touch.  c = 0 (default) picks 6 for state vectors and 4 for
 * density matrices (on vec(rho) a qubit above the low bits needs two high
 * bits, q and q + n, so fewer low bits leave room for more qubits per block);
 * otherwise c in [3, 8], used as max(k - 8, min(c, k - 2)) at width k.  Only
 * the grouping into blocks changes, and results agree to rounding.  Changing
 * it on a DM handle runs the queued superoperators first.  Other values:
 * NWQ_EINVAL. */
int nwq_set_fusion_lowbits(nwq_handle h, int c);

/* Statistics of the last nwq_apply_circuit: number of fused blocks and
 * gates (both 0 when fusion was off). */
int nwq_fusion_stats(nwq_handle h, int* blocks, int* gates);

/* Kernel for fused blocks: 1 (default) = register-blocked with 4 register
 * bits (each thread holds 16 amplitudes over 4 tile bits and applies runs of
 * gates on those bits in registers, one LDS exchange per run), 2 =
 * register-blocked with 3 register bits (8 amplitudes per thread, twice the
 * threads per tile), 0 = one LDS pass per gate.  With 1 or 2, tiles smaller
 * than 2^8 are padded to 2^8 on registers of at least 8 qubits.  Other values:
 * NWQ_EINVAL. */
int nwq_set_fusion_kernel(nwq_handle h, int kernel);
/* Flags of the register-blocked fused kernels (1 and 2): bit 0 = load and
 * store the tiles with non-temporal accesses (each entry is read and written
 * once per block; on the MI355X the depth-40 brickwork at 30 qubits runs
 * about 3% faster with it); bit 1 = when a block's first (last) register
 * phase holds only tile bits above its low contiguous bits, load (store) that
 * phase's registers straight from (to) HBM instead of through LDS; bit 2 =
 * (state vectors, register-blocked kernels) before the blocks are planned, a
 * two-qubit gate and the one-qubit gates next to it on its two qubits, or a
 * run of one-qubit gates on one qubit, become one 4x4 or 2x2 product where
 * that takes fewer FP64 operations (the products round differently: results
 * agree to about 1e-15).
 * Default 7.  Bits 0 and 1 do not change results.  Other values:
 * NWQ_EINVAL. */
int nwq_set_fusion_flags(nwq_handle h, int flags);

/* Number of register phases (LDS exchanges) of the last fused
 * nwq_apply_circuit (0 when no register-blocked block ran). */
int nwq_fusion_phases(nwq_handle h, int* phases);

/* Host-only: the block plan nwq_apply_circuit would use for a circuit on n
 * qubits at fusion width k with gate products off (nwq_set_fusion_flags bit
 * 2 clear; products depend on the gates' parameters, which are not needed
 * here).  Writes the number
 * of blocks to *n_blocks, the block index of each gate to block_of_gate[]
 * (n_gates entries), and, if block_qubits is non-NULL, each block's tile
 * qubit mask as two 32-bit halves (2 * n_gates ints of room).  Touches no
 * device. */
int nwq_fusion_plan(int n, int k, int n_gates, const int* types, const int* qubits,
                    int* n_blocks, int* block_of_gate, int* block_qubits);

/* ---------------------------------------------------------------------------
 * Noise channels (Sec. III noise model; DM handles only, else NWQ_EKIND)
 * ------------------------------------------------------------------------- */

/* rho <- sum_k K_k rho K_k^dag for n_kraus operators of size 2^k x 2^k
 * (k = 1 or 2) given back to back (complex, row-major, interleaved).
 * NWQ_ENOTCPTP if max |sum K^dag K - I| > 1e-12. */
int nwq_apply_channel(nwq_handle h, const int* qubits, int k,
                      const double* kraus, int n_kraus);

/* Depolarising channel on k = 1 or 2 qubits:
 *   rho <- (1 - p) rho + p I/2^k (x) Tr_qubits(rho),  0 <= p <= 1. */
int nwq_depolarize(nwq_handle h, const int* qubits, int k, double p);
/* The same with a choice of convention (the paper names depolarisation
 * without fixing one):
 *   NWQ_DEPOL_REPLACE: as nwq_depolarize;
 *   NWQ_DEPOL_PAULI:   rho <- (1 - p) rho + p / (4^k - 1) sum_{P != I} P rho P
 *                      (uniform Pauli errors of total probability p).
 * The two agree at p_PAULI = p_REPLACE (4^k - 1) / 4^k.  NWQ_EINVAL for
 * another convention value. */
#define NWQ_DEPOL_REPLACE 0
#define NWQ_DEPOL_PAULI 1
int nwq_depolarize_ex(nwq_handle h, const int* qubits, int k, double p, int convention);
/* Amplitude damping: K0 = [[1,0],[0,sqrt(1-g)]], K1 = [[0,sqrt g],[0,0]]. */
int nwq_amp_damp(nwq_handle h, int q, double gamma);
/* Phase damping: K0 = [[1,0],[0,sqrt(1-l)]], K1 = [[0,0],[0,sqrt l]]. */
int nwq_phase_damp(nwq_handle h, int q, double lambda);
/* Thermal relaxation of qubit q over a duration t, from the device
 * calibration values T1 and T2 (Sec. III device noise model): the excited
 * population decays as e^{-t/T1} into |0> and the coherences as e^{-t/T2}.
 * Applied as amplitude damping with gamma = 1 - e^{-t/T1} followed by phase
 * damping with lambda = 1 - e^{-t (2/T2 - 1/T1)} (fused with the pending gate
 * like any channel).  Requires T1 > 0, 0 < T2 <= 2 T1, t >= 0 (NWQ_EINVAL);
 * DM handles only (NWQ_EKIND). */
int nwq_thermal_relax(nwq_handle h, int q, double t1, double t2, double t);

/* ---------------------------------------------------------------------------
 * Observables (Sec. III: magnetisation, energy)
 * ------------------------------------------------------------------------- */

/* out_real = sum_t coeffs[t] * Re <P_t> (SV: <psi|P|psi>, DM: Tr(rho P)).
 * Synchronises.  Deterministic: reductions use a fixed order. */
int nwq_expval_pauli_sum(nwq_handle h, int n_terms, const uint64_t* xmask,
                         const uint64_t* zmask, const double* coeffs,
                         double* out_real);

/* out[t] = Re <P_t> for each term (no coefficients).  Synchronises. */
int nwq_expval_pauli_terms(nwq_handle h, int n_terms, const uint64_t* xmask,
                           const uint64_t* zmask, double* out);
/* As nwq_expval_pauli_terms with imaginary parts: out_real[t] = Re <P_t>,
 * out_imag[t] = Im <P_t> (out_imag may be NULL).  DM: both parts of
 * Tr(rho P_t) as summed by the kernel, so |Im| measures how far the state
 * has drifted from Hermitian.  SV: P_t is Hermitian, so the contributions of
 * the index pairs (j, j ^ x) are complex conjugates; the kernels sum each
 * pair once (twice its real part), and Im <P_t> is 0 by construction and
 * returned as 0.  Synchronises. */
int nwq_expval_pauli_terms_complex(nwq_handle h, int n_terms, const uint64_t* xmask,
                                   const uint64_t* zmask, double* out_real, double* out_imag);

/* Device bytes the handle holds now: the state if the library allocated it
 * (nwq_*_create, not *_create_from), the 4 MiB upload ring once used,
 * reduction scratch and the fused-block program buffer.  Host-side
 * bookkeeping only: no device call. */
int nwq_memory(nwq_handle h, size_t* bytes);

/* DM only: out = Re Tr(rho) (imaginary part in *imag_out if non-NULL). */
int nwq_trace(nwq_handle h, double* out, double* imag_out);
/* DM: sum_jk |rho_jk|^2 (= Tr rho^2 for Hermitian rho); SV: sum |a_j|^2. */
int nwq_purity(nwq_handle h, double* out);

/* ---------------------------------------------------------------------------
 * VQE energies and adjoint gradients (Sec. III, Fig. 4: VQE for the Ising
 * model).  Gradients follow adjoint differentiation (Jones & Gacon,
 * arXiv:2009.02823): one backward sweep of U_k^dag over (phi, H phi).
 * ------------------------------------------------------------------------- */

typedef struct nwq_vqe* nwq_vqe_handle;

/* Build a VQE context for an n-qubit register (1 <= n <= 30) starting from
 * |0...0>.  The program has n_ops gates: types[i] (nwq_gate), qubits[2i],
 * qubits[2i+1] (second entry ignored for 1-qubit gates) and params[i], the
 * index into theta (0 <= params[i] < n_params) for the parametrised types RX,
 * RY, RZ, RZZ (each exp(-i theta P / 2)); params[i] is ignored for the fixed
 * types I X Y Z H S SDG T TDG CX CZ SWAP (U3 is not allowed).  The
 * Hamiltonian is sum_t coeffs[t] P_t over n_terms Pauli strings (xmask,
 * zmask).  Host arrays are copied.  The context owns a HIP stream of its own;
 * evaluations are ordered after prior work on `hip_stream` and later work on
 * `hip_stream` is ordered after them. */
int nwq_vqe_create(int n, int n_ops, const int* types, const int* qubits, const int* params,
                   int n_params, int n_terms, const uint64_t* xmask, const uint64_t* zmask,
                   const double* coeffs, void* hip_stream, nwq_vqe_handle* out);
int nwq_vqe_destroy(nwq_vqe_handle h);
int nwq_vqe_info(nwq_vqe_handle h, int* n_params, int* n_ops, int* n_slots);

/* Device memory of a context, for callers that budget HBM (the serving
 * loop): *held = bytes the context holds now (program tables, the fused-block
 * program once built, and the per-vector buffers of the batched path at its
 * current capacity); *at_B = bytes it will hold after evaluating B vectors
 * with its current configuration (the per-vector buffers grow to the largest
 * B evaluated and are kept until nwq_vqe_destroy; the LDS-resident path
 * needs none; the fused-block program, tens of KiB, is not counted before
 * it is built).  Either pointer may be NULL.  Host-side bookkeeping only:
 * no device call. */
int nwq_vqe_memory(nwq_vqe_handle h, int B, size_t* held, size_t* at_B);

/* Batched path: B parameter vectors theta_dev[B][n_params] (device, FP64)
 * -> energy_dev[B] and, if grad_dev is non-NULL, grad_dev[B][n_params]
 * (device).  n <= 12 runs one persistent LDS-resident kernel (one workgroup
 * per vector); larger n run the fused-block schedule over all B states
 * (see nwq_vqe_set_config), captured once per (B, with/without gradient)
 * into a hipGraph and replayed.  Results for a vector do not depend on B or
 * on the other vectors. */
int nwq_vqe_eval(nwq_vqe_handle h, int B, const double* theta_dev, double* energy_dev, double* grad_dev);

/* As nwq_vqe_eval, with per-vector Hamiltonian coefficients:
 * coeffs_dev[B][n_terms] (device) replaces the context's coefficients for
 * each vector (same Pauli strings).  Used by the serving loop to batch
 * requests whose fields differ. */
int nwq_vqe_eval_coeffs(nwq_vqe_handle h, int B, const double* theta_dev, const double* coeffs_dev,
                        double* energy_dev, double* grad_dev);

/* Plain per-circuit path (the reference point for the batched path): one
 * vector, one kernel per gate, no graph, no LDS residency. */
int nwq_vqe_eval_single(nwq_vqe_handle h, const double* theta_dev, double* energy_dev, double* grad_dev);

/* Launch configuration: mode 0 = automatic (LDS-resident for n <= 12, fused
 * for larger n), 1 = LDS-resident (n <= 12), 2 = one kernel per gate over the
 * batch, 3 = fused blocks (n >= 8: 2^11-amplitude tiles; forward through the
 * register-blocked block kernel over all B states, backward with tiles of phi
 * and lambda in LDS); all but the LDS-resident path run as one hipGraph per
 * batch size.  threads: workgroup size of the LDS kernel (64..1024, power of
 * two); blocks_per_state: workgroups per state of modes 2 and 3 (0 = default). */
int nwq_vqe_set_config(nwq_vqe_handle h, int mode, int threads, int blocks_per_state);
int nwq_vqe_get_config(nwq_vqe_handle h, int* mode, int* threads, int* blocks_per_state);
/* Flags of the fused schedule's tile kernels (forward and backward): bit 0 =
 * non-temporal loads and stores of the tiles; bit 1 = direct HBM loads and
 * stores of a forward block's first and last register phase where the block
 * allows it (as in nwq_set_fusion_flags).  Default 3.  Results do not depend
 * on the flags.  Other values: NWQ_EINVAL. */
int nwq_vqe_set_flags(nwq_vqe_handle h, int flags);
/* Low tile bits of the fused schedule's blocks (mode 3), as
 * nwq_set_fusion_lowbits for circuits: 0 (default) = 3, else c in [3, 8],
 * used as max(k - 8, min(c, k - 2)) at tile width k.  Fewer low bits let a
 * block hold more qubits (n=20, L=8: 26 backward blocks with 6, 18 with 3).
 * Changing it waits for the context's stream and plans the program again
 * on next use.  Results agree to rounding.  Other values: NWQ_EINVAL. */
int nwq_vqe_set_lowbits(nwq_vqe_handle h, int c);

/* Batched VQE for the Ising model of Sec. III (Fig. 4) in one call, without
 * a context: the n-qubit hardware-efficient ansatz of L layers (each layer
 * RY(theta) on qubits 0..n-1, RZ(theta) on 0..n-1, then CX(0,1), CX(1,2), ...,
 * CX(n-2,n-1); P = 2 n L parameters, layer-major, RY block then RZ block)
 * from |0...0>, and the open-chain transverse-field Ising Hamiltonian
 * H = -J sum_{i<n-1} Z_i Z_{i+1} - h sum_i X_i with J = J_h[0], h = J_h[1]
 * (host array of two finite doubles, shared by the batch).
 * theta_dev[B][P] (device, FP64) -> E_dev[B] and, if grad_dev is non-NULL,
 * grad_dev[B][P] (device), exactly as nwq_vqe_eval on a context built with
 * nwq_vqe_create from the same program and terms.  The library keeps one
 * context per (device, n, L), up to 8 (least recently used freed first), so
 * only the first call for a shape allocates; a new (J, h) rewrites the
 * context's term table after its earlier work has finished (the call waits
 * for it).  Ordered on `stream` like nwq_vqe_eval.  1 <= n <= 30, L >= 1,
 * 1 <= B <= 65535; errors before any launch leave the outputs untouched.
 * Calls are serialised by a library lock. */
int nwq_vqe_batch(int n, int L, const double* J_h, int B, const double* theta_dev, double* E_dev, double* grad_dev,
                  void* stream);
/* Frees every context nwq_vqe_batch keeps (waits for their work). */
int nwq_vqe_batch_release(void);

/* Autotuner: times every valid (mode, threads, blocks_per_state) candidate on
 * B zero parameter vectors with HIP events, keeps the fastest and returns
 * its time per batch in *best_ms.  Synchronises. */
int nwq_vqe_autotune(nwq_vqe_handle h, int B, int with_grad, double* best_ms);

/* ---------------------------------------------------------------------------
 * Launch shapes and their autotuner
 * ------------------------------------------------------------------------- */

/* Kernel class ids are the timing classes below (1 sv_1q_dense, 2 sv_diag,
 * 3 sv_perm, 4 sv_2q_dense, 6 dm_superop_1q, 7 dm_superop_2q).
 *
 * A launch shape is the number of pairs / groups per thread (1, 2, 4 or 8;
 * also 16 for classes 1, 2 and 3; class 7 takes 1, 64 and 128 only) and a flags
 * word (the argument named nontemporal).  Bit 0 of the flags puts a
 * non-temporal hint on the loads and stores.  Bit 1, taken with shapes 32,
 * 64 and 128 and with shape 1 of class 2, orders the workgroups so that each
 * of the chip's 8 XCDs streams one contiguous eighth of the launch: workgroup
 * i takes block (i mod 8) G/8 + floor(i / 8) of G (launches whose G is not a
 * multiple of 8 keep dispatch order).  Other flags are NWQ_EINVAL.
 *
 * Shapes 32, 64 and 128 select split-workgroup kernels of 256, 512 or 1024
 * threads, one entry per thread:
 *  - class 1, targets from 9 up: the lower members of the workgroup's pairs
 *    in one half, the upper members in the other, exchanged through LDS
 *    (targets 0..8 always use an LDS partner exchange, with the flags only);
 *  - class 3: X, CX and SWAP with the two moved members of a group in the two
 *    halves, each written to its partner's place after a barrier (gates whose
 *    bits are all lane bits keep their lane exchange, one entry per thread);
 *  - classes 4 and 6 (4x4 operators): a quarter of the workgroup holds each
 *    member of its quads and each thread forms one row of the operator from
 *    LDS (operators with one bit below 3 and the other at or above 6 keep
 *    their lane exchange);
 *  - class 7, shapes 128 and 64: each of the 16 waves of a 1024-thread
 *    workgroup holds one member of 64 groups (128), or each of the 8 waves
 *    of a 512-thread workgroup holds two (64), and the 16 x 16 operator is
 *    applied the same way (low-qubit operators that fit the LDS-staged
 *    kernel keep it).
 *
 * Each class keeps one shape per bucket of the launch's lowest target bit:
 * bucket 0 for bits 0..2 (partner amplitudes in one 128-byte line), 1 for
 * bits 3..10, 2 for bits 11 and up.  nwq_set_launch with bucket -1 sets all
 * three. */
#define NWQ_LAUNCH_BUCKETS 3
int nwq_set_launch(nwq_handle h, int cls, int bucket, int ppt, int nontemporal);
int nwq_get_launch(nwq_handle h, int cls, int bucket, int* ppt, int* nontemporal);

/* Per-target shapes: a launch whose lowest target bit is `bit` (0..63) uses
 * the shape set for that bit, if any, else its bucket's.  nwq_set_launch
 * clears the per-target shapes of the buckets it sets; ppt 0 here clears one.
 * nwq_get_launch_target returns the shape a launch on that bit would use. */
#define NWQ_LAUNCH_TARGET_BITS 64
int nwq_set_launch_target(nwq_handle h, int cls, int bit, int ppt, int nontemporal);
int nwq_get_launch_target(nwq_handle h, int cls, int bit, int* ppt, int* nontemporal);

/* Autotuner: for each class that applies to the handle (SV: 1, 2, 3, 4;
 * DM: 6, 7) and each lowest target bit, time every launch shape with HIP
 * events on the handle's stream and state (self-inverse operations whose
 * entries are 0 or +-1, applied in pairs: every product and sum is exact, so
 * the state's values are unchanged).  Each target
 * bit keeps its fastest shape; each bucket keeps the shape with the least
 * total time over its bits.  The mean over a bucket's bits of their best time
 * per launch (ms) goes to best_ms[class * NWQ_LAUNCH_BUCKETS + bucket]
 * (NWQ_TIMING_CLASSES * NWQ_LAUNCH_BUCKETS entries, -1 where not tuned;
 * best_ms may be NULL).  Flushes deferred work first; synchronises. */
int nwq_autotune(nwq_handle h, int reps, double* best_ms);

/* Fusion autotuner (SV handles): runs the given circuit (arrays as for
 * nwq_apply_circuit) from |0...0> as nwq_run_circuit does (the reset
 * included) once untimed and reps times timed under
 * each candidate: unfused, and every fusion width from 6 to min(13, n) with
 * each fused kernel (the register-blocked ones only on 8 or more qubits).
 * Keeps the fastest on the handle and returns it in *best_k (0 = unfused)
 * and *best_rb (the nwq_set_fusion_kernel value).  If ms_out is non-NULL it
 * receives NWQ_FUSION_CANDIDATES times in ms per circuit (-1 for candidates
 * not run): index 0 unfused, 1 + 3 * (k - 6) + kernel for width k.
 * Overwrites the state and leaves it at |0...0>; synchronises. */
#define NWQ_FUSION_CANDIDATES 25
int nwq_autotune_fusion(nwq_handle h, int n_gates, const int* types, const int* qubits,
                        const double* params, int reps, int* best_k, int* best_rb, double* ms_out);

/* ---------------------------------------------------------------------------
 * Measurement: outcome probabilities, readout noise, shot sampling
 * (provider semantics of Sec. II; measurement noise of the Sec. III device
 * noise model).  Outcome j is the basis index (qubit q = bit q of j).
 * ------------------------------------------------------------------------- */

/* probs_dev[j] = |a_j|^2 (SV) or Re rho_jj (DM) for j < 2^n: a caller-owned
 * device array of 2^n doubles.  Flushes deferred work, then runs
 * asynchronously on the handle's stream. */
int nwq_probabilities(nwq_handle h, double* probs_dev);

/* Readout noise on an outcome distribution of 2^n doubles (device, in
 * place): for each qubit q a confusion matrix C_q with
 * C_q[r][t] = P(read r | true t), given as confusion[4q .. 4q+3] =
 * C[0][0], C[0][1], C[1][0], C[1][1]; p <- (C_{n-1} (x) ... (x) C_0) p.
 * Entries must lie in [0, 1] and each column sum to 1 (within 1e-12), else
 * NWQ_EINVAL before any launch.  Identity matrices are skipped; the others
 * run up to five qubits per pass.  Asynchronous on `stream` (hipStream_t). */
int nwq_readout_noise(int n, double* probs_dev, const double* confusion, void* stream);

/* Workspace of nwq_sample in bytes (0 if n is outside [1, 34]). */
size_t nwq_sample_workspace_bytes(int n);

/* Shot sampling from an outcome distribution of 2^n doubles (device; the
 * entries should sum to 1 and must sum to at most 4).  Each p_j is quantised
 * to q_j = floor(p_j 2^61) (p_j <= 0 or NaN gives 0, p_j >= 1 gives 2^61);
 * the inclusive integer CDF C_j = q_0 + ... + q_j is built in work_dev
 * (its first 2^n uint64 entries, left there for the caller); shot s with
 * uniform u_dev[s] in [0, 1) returns out_dev[s] = the smallest j with
 * C_j > floor(floor(u 2^53) Q / 2^53), Q = C_{2^n-1} (-1 if Q = 0).  u is
 * clamped into [0, 1 - 2^-53].  work_bytes must be at least
 * nwq_sample_workspace_bytes(n).  0 <= shots < 2^31.  Asynchronous on
 * `stream`.  The result depends on the inputs only (exact integer sums). */
int nwq_sample(int n, const double* probs_dev, const double* u_dev, long long shots, long long* out_dev,
               void* work_dev, size_t work_bytes, void* stream);

/* Allocation-free variant of nwq_sample, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments and results as nwq_sample, bit for
 * bit, without the workspace: the CDF, tile totals and tile offsets live in a
 * device array inside the library (8 MiB per GPU, held until the process
 * ends), so n must be at most 20 (NWQ_ERANGE otherwise, before any launch).
 * The call allocates nothing (its first call on a device looks up that
 * device's array once).  Every call on one GPU shares that GPU's array and
 * overwrites it: calls that overlap on one GPU (different streams or
 * threads) race, and must be ordered by the caller.  The stream must belong
 * to the current device.  Asynchronous on `stream`. */
int nwq_sample_noalloc(int n, const double* probs_dev, const double* u_dev, long long shots, long long* out_dev,
                       void* stream);

/* ---------------------------------------------------------------------------
 * Diagnostics
 * ------------------------------------------------------------------------- */

/* Message of the last failed call on this thread ("" if none). */
const char* nwq_last_error(void);

/* Streaming ceilings (yardsticks for the gate kernels' bandwidth): an
 * in-place scale a_j <- s a_j of n_entries complex128 entries (read and
 * write at the same address, the access pattern of a gate pass), and a copy
 * dst_j <- src_j (buffers must not overlap).  One entry per thread with
 * non-temporal loads and stores, workgroups in XCD-contiguous order.
 * Asynchronous on `stream` (hipStream_t); NWQ_EINVAL on a NULL buffer. */
int nwq_stream_scale(void* buf_dev, size_t n_entries, double s, void* stream);
int nwq_stream_copy(void* dst_dev, const void* src_dev, size_t n_entries, void* stream);

/* Per-kernel timing with HIP events on the handle's stream: when enabled,
 * every launch is bracketed by events and nwq_timing_read returns, per
 * kernel class, the number of launches and the summed milliseconds since
 * the last reset (it synchronises).  Classes: 0 reset, 1 sv_1q_dense,
 * 2 sv_diag, 3 sv_perm, 4 sv_2q_dense, 5 sv_fused, 6 dm_superop_1q,
 * 7 dm_superop_2q, 8 reduce.  count and ms hold NWQ_TIMING_CLASSES entries. */
#define NWQ_TIMING_CLASSES 9
int nwq_timing_enable(nwq_handle h, int enable);
int nwq_timing_read(nwq_handle h, long long* count, double* ms, int reset);

#ifdef __cplusplus
}
#endif

#endif /* NWQ_H */
