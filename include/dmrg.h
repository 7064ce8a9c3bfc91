/*
 * dmrg.h - C ABI of the MI355X two-site shell-model DMRG hot path.
 *
 * Method (Legeza, Veis, Poves, Dukelsky, arXiv:1507.00161):
 *   H = sum_a eps_a c+_a c_a + two-body term            (Eq. 1)
 * on m-scheme single-particle sites a = (n, l, j, m, tau_z), each empty or
 * occupied (the C^2 representation, local dimension 2).  The state is
 * optimised on a two-site superblock  Xi(l) x Lambda x Lambda x Xi(r)  of an
 * ordered orbital chain, the block bases are truncated to D states through
 * the Schmidt (SVD) decomposition of the superblock state, and the chain is
 * swept back and forth (the two-site DMRG paragraph and the block-state
 * paragraph that introduces M, called D here).  The conserved quantities are
 * the proton and neutron numbers and the total J_z (the m-scheme basis
 * dimension "for J_z = 0").
 *
 * This library runs one GPU (gfx950).  All device work is issued on the
 * context stream; calls on one context must not overlap (one host thread at
 * a time per context); different contexts are independent.  Nothing throws or
 * aborts across this boundary: every call returns a dmrg_status and stores a
 * message retrievable with dmrg_last_error.
 */
#ifndef DMRG_MI355X_H
#define DMRG_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dmrg_status {
    DMRG_OK = 0,
    DMRG_WARN_NOT_CONVERGED = 1,   /* a Davidson solve hit davidson_max_iter; results valid */
    DMRG_ERR_ARG = -1,             /* invalid argument (null pointer, D < 1, bad ordering, ...) */
    DMRG_ERR_HAMILTONIAN = -2,     /* eps / V violate a symmetry or selection rule */
    DMRG_ERR_TARGET = -3,          /* (n_p, n_n, 2M) not reachable in the space */
    DMRG_ERR_STATE = -4,           /* call out of order (e.g. apply before any sweep) */
    DMRG_ERR_OUT_OF_MEMORY = -5,   /* device allocation failed or mem_cap_bytes exceeded */
    DMRG_ERR_DEVICE = -6           /* HIP / library error */
} dmrg_status;

typedef enum dmrg_precision {
    DMRG_FP64 = 0,        /* every H_eff.psi sector GEMM in FP64 */
    DMRG_MIXED_FP32 = 1,  /* Davidson expansion products in FP32, FP64 residual correction */
    DMRG_MIXED_BF16 = 2   /* BF16 inputs with FP32 accumulation, FP64 residual correction */
} dmrg_precision;

typedef struct dmrg_options {
    int32_t precision;             /* dmrg_precision, default DMRG_FP64 */
    uint64_t seed;                 /* key of the hash-random start, default 1507 */
    double davidson_tol;           /* residual 2-norm (MeV) for convergence, default 1e-7 */
    int32_t davidson_max_iter;     /* H_eff products per solve, default 100 */
    int32_t davidson_max_subspace; /* subspace size before restart, default 24 (<= 32) */
    double noise;                  /* density-matrix perturbation weight, default 0 */
    int32_t noise_sweeps;          /* sweeps (from the start) that use `noise`, default 0 */
    int32_t select_basis;          /* 1: truncate by determinant selection (test mode) */
    double tie_tol;                /* truncation tie tolerance on weights, default 1e-13 */
    int32_t device;                /* HIP device ordinal, default 0 */
    void* stream;                  /* hipStream_t to use, NULL = context-owned stream */
    uint64_t mem_cap_bytes;        /* 0 = no cap; else device bytes the context may hold */
    uint64_t scratch_bytes;        /* 0 = automatic; else cap on H_eff intermediate buffers */
    /* Dynamic block-state selection (DBSS, the paper's block-state paragraph
     * after Eq. 1): with trunc_eps > 0 each truncation keeps the fewest
     * largest density-matrix weights whose discarded remainder
     * 1 - sum(kept), summed in descending order, is at most trunc_eps, and
     * then at least d_min and at most the sweep's D states; the tie rule
     * applies to that count.  trunc_eps = 0 (default): D states. */
    double trunc_eps;              /* default 0; must be >= 0 */
    int32_t d_min;                 /* default 0; must be >= 0 */
    /* 1 (default): the ground state.  2: the two lowest states targeted at
     * once (the paper's excitation-energy paragraph): at each bond the second
     * state is the lowest eigenpair of H_eff orthogonal to the first (a
     * Davidson solve in its complement), both are predicted to the next bond,
     * and the truncation uses their density matrices averaged with equal
     * weights.  dmrg_energy, dmrg_heff_layout/apply and dmrg_get_psi refer to
     * the first state; the second state's energy is in the sweep statistics. */
    int32_t n_states;
    /* 1: measure the orbital correlations of the (first) state during the
     * right-to-left half of every sweep, for the one-orbital entropies and the
     * two-orbital mutual information of the paper's entropy paragraph
     * (dmrg_orbital_entropies).  At bond b the state gives <n_j>, and for every
     * i <= b <n_i>, <n_i n_j> and <c+_i c_j>, with j = b + 1.  Left blocks then
     * carry the occupation operator of each of their sites.  0 (default): off. */
    int32_t measure;
    /* 1: each bond's H_eff product (input and output conversions, the GEMM
     * phases, their split-K reductions) is captured once in a HIP graph and
     * the graph is replayed for every product at that bond (input and output
     * pass through fixed staging vectors).  Products then run as one graph
     * launch; the per-phase GEMM statistics are not collected.  Products that
     * need several term groups, and products of contexts advanced by
     * dmrg_sweep_many, are launched directly.  0 (default): direct launches. */
    int32_t graph;
    /* dmrg_sweep_many only: 1 (default) = when every context of the call has
     * 1 and all are on one device, their H_eff products are launched in
     * groups (one grouped persistent-GEMM launch per phase over all pending
     * products); 0 = each context launches its own products on its own
     * stream, and the device runs the contexts' kernels concurrently. */
    int32_t group_products;
} dmrg_options;

typedef struct dmrg_sweep_stats {
    double energy;            /* lowest step energy of the sweep (MeV) */
    double last_theta;        /* energy at the last step */
    double discarded_max;     /* largest discarded weight 1 - sum(kept) */
    double discarded_sum;
    int64_t products_low;     /* H_eff.psi products in reduced precision */
    int64_t products_fp64;    /* H_eff.psi products in FP64 */
    int64_t solves;           /* Davidson solves */
    int64_t not_converged;    /* solves that hit davidson_max_iter */
    double heff_flops;        /* algorithmic flops of all H_eff.psi products */
    double heff_seconds;      /* device time of all H_eff.psi products (HIP events) */
    double sweep_seconds;     /* wall time of the sweep */
    /* Host wall time of the stages below.  Device work is queued without
     * waiting where nothing on the host needs its result, so a stage's time
     * includes device work only up to the waits it makes (the eigenvalue read
     * of the truncation, the norm check of the prediction). */
    double renorm_seconds;    /* truncation + renormalisation + prediction (incl. blocking) */
    double blocking_seconds;  /* building enlarged-block operators and plans */
    double density_seconds;   /* of renorm_seconds: reduced density matrices */
    double eig_seconds;       /* of renorm_seconds: sector eigendecompositions + selection */
    double renormalize_seconds; /* of renorm_seconds: U^T O U of the kept operators */
    double predict_seconds;   /* of renorm_seconds: next-bond guess */
    int32_t status;           /* per-context status (dmrg_sweep_many) */
    int32_t steps;            /* two-site steps done */
    /* per-kernel accounting of the H_eff.psi grouped GEMMs (HIP events on the
     * context stream): phase 1 (kernel k_heff_z) forms psi op(B)^T, phase 2
     * (k_heff_y) accumulates op(A) Z.  Only launches in the context's working
     * precision are counted (FP64 in DMRG_FP64 mode, the reduced precision in
     * the mixed modes); the split-K reduction after phase 2 is timed apart. */
    int64_t gemm1_launches, gemm2_launches;
    double gemm1_seconds, gemm2_seconds;
    double gemm1_flops, gemm2_flops;
    double gemm1_bytes, gemm2_bytes;   /* algorithmic operand + result bytes */
    double reduce_seconds;             /* split-K reductions of those launches */
    int64_t kept_max;                  /* most block states kept by a truncation of the sweep */
    double energy_excited;             /* n_states = 2: lowest step energy of the second state (MeV) */
    double measure_seconds;            /* measure = 1: host wall time of the correlation measurements */
    /* heff_flops counts, per product, for every term and psi block the
     * cheaper of the two contraction orders (op(A) psi first, or psi op(B)^T
     * first) over the nonzero sub-sector blocks of the operators, with true
     * block dimensions and each intermediate formed once.  The kernels run the
     * psi op(B)^T-first order; heff_flops_executed is what they multiply over
     * columns that can be nonzero, and gemm{1,2}_flops split it by phase.
     * gemm{1,2}_issued_flops also count the cleared columns that phase 2
     * multiplies when it spans an output block's full width. */
    double heff_flops_executed;
    double gemm1_issued_flops, gemm2_issued_flops;
    /* dmrg_check_fp64 on: solves repeated in FP64 from the same guess, and the
     * largest |theta - theta_fp64| / |theta_fp64| over them */
    int64_t check_solves;
    double check_max_rel;
    /* energy minus that of the previous full sweep of this context (MeV);
     * NaN for the first sweep after the blocks were set up (first call, new
     * ordering, reloaded Hamiltonian) and for statistics of an unfinished
     * sweep.  The paper stops sweeping once |delta_energy| < 1e-4 MeV. */
    double delta_energy;
} dmrg_sweep_stats;

typedef struct dmrg_ctx dmrg_ctx;

/* Fill `opt` with the defaults listed above. */
void dmrg_default_options(dmrg_options* opt);

/* Create a context on opt->device (NULL opt = defaults).  *out owns all its
 * device memory; release with dmrg_destroy.  Errors: ARG, DEVICE. */
dmrg_status dmrg_create(const dmrg_options* opt, dmrg_ctx** out);
void dmrg_destroy(dmrg_ctx* ctx);

/* Hamiltonian of Eq. 1 on n_sites m-scheme sites, written
 *   H = sum_i eps_i n_i + 1/4 sum_ijkl V_ijkl c+_i c+_j c_l c_k
 * (host arrays, copied; the caller keeps ownership):
 *   species[n]  0 = proton, 1 = neutron;  two_m[n]  twice the m projection;
 *   eps[n] MeV; V[n*n*n*n] row-major V[((i*n+j)*n+k)*n+l], antisymmetrised.
 * Validation (tolerance 1e-12 * max|V|): V_ijkl = -V_jikl = -V_ijlk = V_klij,
 * and V_ijkl = 0 unless 2m_i+2m_j = 2m_k+2m_l and {tau_i,tau_j} = {tau_k,tau_l}
 * -> DMRG_ERR_HAMILTONIAN naming the first offending (i,j,k,l).
 * Target (n_p, n_n, 2M): DMRG_ERR_TARGET if no determinant has it.
 * Reloading resets all DMRG state.  1 <= n_sites <= 64. */
dmrg_status dmrg_load_hamiltonian(dmrg_ctx* ctx, int32_t n_sites, const int32_t* species,
                                  const int32_t* two_m, const double* eps, const double* V,
                                  int32_t n_p, int32_t n_n, int32_t two_M);

/* One sweep: left-to-right over bonds 0..N-2 then right-to-left back to 0,
 * keeping at most D block states.  `ordering` (host, a permutation of
 * 0..N-1; NULL = natural order) maps chain position -> site.  The first call,
 * or a call with a different ordering, (re)initialises the blocks; D may
 * change between calls.  `out` (nullable) receives the sweep statistics.
 * Returns DMRG_WARN_NOT_CONVERGED if a Davidson solve hit its limit. */
dmrg_status dmrg_sweep(dmrg_ctx* ctx, const int32_t* ordering, int32_t D, dmrg_sweep_stats* out);

/* Advance at most n_steps two-site steps of the sweep schedule (a full sweep
 * is 2(N-1) steps), continuing from where the previous call stopped. */
dmrg_status dmrg_sweep_steps(dmrg_ctx* ctx, const int32_t* ordering, int32_t D, int32_t n_steps,
                             dmrg_sweep_stats* out);

/* Layout of psi at the current bond (sites bond, bond+1 explicit).  psi is a
 * list of dense row-major blocks, one per S sector q (S = chain sites
 * 0..bond), in ascending (n_p, n_n, 2M) order; block q has
 * sector_dims[2s] rows (S states: site `bond` empty part first) and
 * sector_dims[2s+1] columns (E states of sector target - q: site `bond+1`
 * empty part first).  Call with NULL arrays to get n_sectors first. */
dmrg_status dmrg_heff_layout(dmrg_ctx* ctx, int32_t* bond, int64_t* dim, int32_t* n_sectors,
                             int32_t* sector_qn, int64_t* sector_dims);

/* y = H_eff psi at the current bond (the superblock Hamiltonian P^T H P in
 * the current block bases).  psi_in, psi_out: device pointers, FP64, `dim`
 * elements in the dmrg_heff_layout order, caller-owned, must not overlap.
 * The sector GEMMs run in `precision` (dmrg_precision); I/O stays FP64.
 * Asynchronous on the context stream; synchronise the stream before reading.
 * DMRG_ERR_STATE before the first sweep step. */
dmrg_status dmrg_heff_apply(dmrg_ctx* ctx, const double* psi_in, double* psi_out, int32_t precision);

/* CI-DEAS start (the block-state paragraph: the environmental error of the
 * first sweeps is reduced by a CI-based, dynamically extended active space
 * grown by the orbital entropy profile).  s1[n_sites] and n1[n_sites] (host,
 * site indices, copied) are the one-orbital entropies and occupations <n_i>
 * of a preprocessing run (dmrg_orbital_entropies of a measuring sweep).  The
 * next sweep re-initialises: every environment block R = chain positions
 * lo..N-1 keeps determinants of its composite basis (position lo times the
 * block built before it): those that differ from the reference determinant
 * (per species the sites of largest <n_i>, ties to the lower position) only
 * on the block's k most entropic positions, for the largest k whose CI space
 * holds at most D of them, completed to D from the next space with the
 * fewest differing positions first, then the SplitMix64 key
 * (seed, 5, lo, low and high 32 bits of the determinant as a chain-position
 * mask).  The first state is the hash-random vector.  Both NULL: back to the
 * hash start (also re-initialising).  Reloading the Hamiltonian clears it.
 * Errors: STATE before dmrg_load_hamiltonian; ARG for one NULL array, or
 * values not finite, entropies below 0 or occupations outside [0, 1] (by
 * more than 1e-9: measured values carry rounding, and only their order
 * matters). */
dmrg_status dmrg_set_cideas(dmrg_ctx* ctx, const double* s1, const double* n1);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as dmrg_heff_apply (same plans, kernels and launch order, so the
 * same result), with every intermediate in a fixed device array of 64 MiB
 * that the library holds on each GPU it runs on until the process ends:
 * the reduced-precision operator copies (converted on every call), the
 * reduced-precision input and output, the intermediate psi op(B)^T and the
 * split-K partial tiles.  No device memory is allocated or freed.  A bond
 * whose intermediates exceed the array returns DMRG_ERR_OUT_OF_MEMORY (with
 * the size needed in dmrg_last_error) and launches nothing.  All calls on a
 * GPU share its array and nothing is carried from one call to the next:
 * calls whose streams can overlap on one GPU (two contexts with different
 * streams) race and must be ordered by the caller.  Arguments, layout and
 * other errors as for dmrg_heff_apply; asynchronous on the context stream. */
dmrg_status dmrg_heff_apply_noalloc(dmrg_ctx* ctx, const double* psi_in, double* psi_out, int32_t precision);

/* Diagnostic for the mixed modes (the FP64 residual correction).  While
 * `on` is 1, every Davidson solve of a mixed-precision context is repeated
 * from the same guess with FP64 products only, on the same H_eff; the repeat's
 * vector is discarded, so the run continues exactly as without the check.
 * The sweep statistics then report the number of such pairs (check_solves)
 * and the largest relative difference of their energies (check_max_rel).
 * The repeats add device time to the sweep (not to heff_seconds).  Ignored
 * in DMRG_FP64 mode.  Errors: ARG for `on` other than 0 or 1. */
dmrg_status dmrg_check_fp64(dmrg_ctx* ctx, int32_t on);

/* FP64 sweep energy (MeV) of the last completed sweep.  DMRG_ERR_STATE before. */
dmrg_status dmrg_energy(dmrg_ctx* ctx, double* E);

/* Current superblock state (host copy, dmrg_heff_layout order). */
dmrg_status dmrg_get_psi(dmrg_ctx* ctx, double* psi_host);

/* Test support: with select_basis = 1 every block state is one determinant;
 * configs[x] (host, dim entries) receives the determinant of psi component x
 * as a bit mask over chain positions (bit a = site ordering[a]); the state is
 * prod_{a in mask, ascending} c+_{ordering[a]} |0>.  DMRG_ERR_STATE otherwise. */
dmrg_status dmrg_heff_configs(dmrg_ctx* ctx, uint64_t* configs);

/* Advance n distinct contexts by one sweep each with their own ordering
 * (orderings[i] may be NULL) and D[i] (independent solves, e.g. many small
 * Hamiltonians).  Each context is driven by a host thread of its own (at most
 * 16 threads; further contexts wait for a free one).  When all contexts are
 * on one device and have group_products = 1, their H_eff products are
 * launched together by one launcher thread: the products pending when it takes them (those that arrived while
 * the previous group was launched) form one grouped launch of the persistent
 * GEMM per product phase over all their plans, and one grouped split-K
 * reduction, on a stream of the call; each context's own work stays on its
 * stream, ordered around those launches by events.  Every result equals that of a separate
 * dmrg_sweep (same plans and arithmetic).  Bonds whose product needs several
 * term groups (larger than the scratch limit) are launched by their context.
 * Per-context status in out[i].status (out may be NULL); returns the first
 * error in context order, else the largest warning.  A NULL or repeated
 * context -> DMRG_ERR_ARG before any work. */
dmrg_status dmrg_sweep_many(dmrg_ctx** ctxs, int32_t n, const int32_t* const* orderings,
                            const int32_t* D, dmrg_sweep_stats* out);

/* One- and two-orbital entropies of the last sweep run with measure = 1
 * (the entropy paragraph).  An orbital is a site (one m-state).  With the
 * proton and neutron numbers and 2M fixed, rho_i = diag(1 - <n_i>, <n_i>)
 * and rho_ij, in the basis |00>, |01>, |10>, |11> of (n_i, n_j), holds
 * <(1-n_i)(1-n_j)>, <(1-n_i) n_j>, <n_i (1-n_j)>, <n_i n_j> on the diagonal
 * and <c+_i c_j> between |01> and |10>.  s = -Tr rho ln rho, and the mutual
 * information is I_ij = s_i + s_j - s_ij (>= 0; the paper prints the
 * opposite sign), all of a pair's values taken from the state at bond j - 1
 * of the chain.  Host outputs, in site indices (the order of
 * dmrg_load_hamiltonian, whatever the chain ordering):
 *   s1[n_sites]                  one-orbital entropies (may be NULL)
 *   mutual[n_sites * n_sites]    I, row-major, symmetric, zero diagonal (may be NULL)
 *   n1[n_sites]                  <n_i> (may be NULL)
 *   nn[n_sites * n_sites]        <n_i n_j>, symmetric, <n_i> on the diagonal (may be NULL)
 *   hop[n_sites * n_sites]       <c+_i c_j> with the Jordan-Wigner order of the
 *                                chain, symmetric, zero diagonal (may be NULL)
 * DMRG_ERR_STATE if no sweep with measure = 1 has completed since the
 * Hamiltonian or the ordering last changed. */
dmrg_status dmrg_orbital_entropies(dmrg_ctx* ctx, double* s1, double* mutual, double* n1, double* nn,
                                   double* hop);

/* Entropy-based ordering (the entropy paragraph, eta = 2): the chain order
 * that sorts the sites by the Fiedler vector, the eigenvector of the second
 * smallest eigenvalue of the Laplacian L = diag(sum_j I_ij) - I of the n x n
 * row-major mutual-information matrix `mutual` (host).  That vector minimises
 * sum_ij I_ij (x_i - x_j)^2 over real x of unit norm orthogonal to the
 * constants, the relaxation of sum_ij I_ij |p_i - p_j|^2 over chain
 * positions p.  Its sign is fixed so that the first nonzero component (in
 * site order) is negative; equal components keep site order.  Writes the
 * permutation ordering[n] (chain position -> site), usable as the ordering
 * of dmrg_sweep; *fiedler_value (may be NULL) receives the eigenvalue.  Host
 * only (cyclic Jacobi); needs no context or device.  Errors: DMRG_ERR_ARG
 * for n < 1, NULL pointers, or a matrix that is not finite and symmetric. */
dmrg_status dmrg_fiedler_ordering(const double* mutual, int32_t n, int32_t* ordering, double* fiedler_value);

const char* dmrg_status_string(dmrg_status s);
const char* dmrg_last_error(const dmrg_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
