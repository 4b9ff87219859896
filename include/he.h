/*
 * he.h — C ABI of the MI355X (gfx950) RNS-CKKS hot path under FHEON's
 * encrypted CNN layers (arXiv 2510.03996).
 *
 * The paper's layers (Section "Secure Neural Network Layers") are built from
 * CKKS slot rotations, plaintext-ciphertext products, additions and rescaling
 * over R_Q = Z_Q[X]/(X^N + 1) in RNS form (Section "Background", CKKS scheme,
 * which also names hoisted "fast rotations").  This library implements that
 * ciphertext arithmetic on the GPU: negacyclic NTT/iNTT, Galois automorphisms,
 * hybrid key switching (ModUp -> key inner product -> ModDown),
 * relinearization, rescale, pt-ct multiply-accumulate, and the layer
 * schedules (conv2d, average pooling, global average pooling, fully
 * connected) on top of them.
 *
 * Data format (all device memory is caller-owned unless stated otherwise):
 *  - Residues are uint64 in [0, q).  A limb holds N residues in NTT form:
 *    index j stores a(psi^(2 brv(j) + 1)) mod q, psi the minimum primitive
 *    2N-th root of unity mod q (bit-reversed evaluation order).
 *  - Moduli are numbered 0..L-1 for the ciphertext primes q_i (q_0 first,
 *    rescale drops the highest active index) and L..L+K-1 for the special
 *    primes p_k of hybrid key switching.
 *  - A ciphertext at level l (l active limbs q_0..q_{l-1}) is he_ct:
 *    `data` points to [2][cap][N] uint64 (c0 limbs at data, c1 limbs at
 *    data + cap*N), cap >= l.
 *  - A plaintext is he_pt: [level][N] uint64 in NTT form; operations use its
 *    first l limbs.
 *  - An evaluation key is [dnum][2][L+K][N] uint64 in NTT form: for digit j
 *    (alpha consecutive Q limbs), poly 0 is b_j and poly 1 is a_j with
 *    b_j = -a_j s + e_j + [P]_{q_i} s' on the digit's limbs and -a_j s + e_j
 *    elsewhere (a key from s' to s; s' = phi_g(s) for a rotation, s^2 for
 *    relinearization).  dnum = ceil(L / alpha).
 *
 * Conventions: every call returns HE_OK (0) or a negative HE_E* code and
 * never throws; he_last_error() gives a thread-local message.  Work is
 * enqueued asynchronously on the given HIP stream (NULL = default stream);
 * host-side scale/level fields of output structs are written before return.
 * Outputs must not alias inputs unless a call says so.
 */
#ifndef HE_H_
#define HE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HE_OK 0
#define HE_EINVAL (-1)       /* bad argument, shape or aliasing */
#define HE_ENOKEY (-2)       /* evaluation key not resident */
#define HE_ELEVEL (-3)       /* level mismatch or exhausted */
#define HE_ESCALE (-4)       /* scale mismatch in an addition */
#define HE_ENOMEM (-5)       /* device allocation failed */
#define HE_EHIP (-6)         /* HIP runtime error */
#define HE_EUNSUPPORTED (-7) /* valid request this library does not implement */

#define HE_MAX_Q 60
#define HE_MAX_P 16
#define HE_KEY_RELIN ((int32_t)0x7fffffff) /* key id of the relinearization key */
/* key id of the conjugation key (Galois element 2N - 1: every slot becomes
 * its complex conjugate); he_rotate with r = HE_KEY_CONJ conjugates */
#define HE_KEY_CONJ ((int32_t)0x7ffffffe)

typedef struct he_ctx he_ctx;
typedef void* he_stream; /* hipStream_t */

/* CKKS parameters.  Primes are either given (q[i], p[k] non-zero) or chosen
 * by the rule: for bit size b the largest not-yet-taken prime q = k 2N + 1
 * with 2^(b-1) < q < 2^b, allocated in the order q_0, q_1..q_{L-1}, p_0..
 * (the paper fixes only bit sizes; Section "HE Security Parameters").
 * Every prime must be < 2^61 and = 1 mod 2N. */
typedef struct {
  int32_t log_n;            /* N = 2^log_n, 12 <= log_n <= 16 */
  int32_t n_q;              /* L, 1..HE_MAX_Q */
  int32_t n_p;              /* K, 1..HE_MAX_P */
  int32_t alpha;            /* Q limbs per key-switching digit; alpha <= K */
  int32_t q_bits[HE_MAX_Q]; /* used when q[i] == 0 */
  int32_t p_bits[HE_MAX_P]; /* used when p[k] == 0 */
  uint64_t q[HE_MAX_Q];
  uint64_t p[HE_MAX_P];
} he_params;

typedef struct {
  uint64_t* data; /* device [2][cap][N] */
  int32_t level;  /* active limbs l */
  int32_t cap;    /* limb capacity per polynomial */
  double scale;   /* CKKS scaling factor carried with the ciphertext */
} he_ct;

typedef struct {
  const uint64_t* data; /* device [level][N] */
  int32_t level;
  double scale;
} he_pt;

/* ------------------------------------------------------------ context */
/* Create a context on `device`: chooses primes, builds twiddle / basis-
 * conversion tables and a workspace pool in device memory (owned by the
 * library until he_ctx_destroy).  HE_EINVAL for unsupported parameters. */
int he_ctx_create(const he_params* params, int device, he_ctx** out);
int he_ctx_destroy(he_ctx* ctx);
/* Copy the L + K moduli (q_0..q_{L-1}, p_0..p_{K-1}) to host `out`. */
int he_ctx_moduli(const he_ctx* ctx, uint64_t* out, int cap);
int he_ctx_info(const he_ctx* ctx, int32_t* log_n, int32_t* n_q, int32_t* n_p, int32_t* alpha);
/* NTT autotuning done at context creation: forward+inverse transforms of
 * 8, 16, 32 and 64 limbs are timed with each of the HE_NTT_VARIANTS kernel
 * shapes (he_ntt_variant); each batch-size bucket (<= 8, <= 16, <= 32,
 * larger limb counts) uses its fastest.  variant[4] (may be NULL) receives
 * the chosen variant per bucket and us[HE_NTT_VARIANTS][4] (may be NULL)
 * the timings in microseconds [variant][bucket]. */
#define HE_NTT_VARIANTS 5
int he_ctx_ntt_tuning(const he_ctx* ctx, int32_t* variant, float* us);
/* Shape of NTT variant v (0 <= v < HE_NTT_VARIANTS): residues staged in LDS
 * per workgroup (`tile`) and residues each thread keeps in registers per LDS
 * round (`per_thread`).  HE_EINVAL for an unknown variant. */
int he_ntt_variant(int v, int32_t* tile, int32_t* per_thread);
/* Replace the autotuned choice: variant[4] gives the variant for each
 * batch-size bucket (for example a choice saved from he_ctx_ntt_tuning, so
 * that runs use identical kernels).  Affects later calls on every stream;
 * do not call while work of this context is being enqueued.  HE_EINVAL for
 * an unknown variant (nothing is changed then). */
int he_ctx_ntt_select(he_ctx* ctx, const int32_t* variant);
/* Basis-conversion tuning done at context creation.  The conversion of
 * hybrid key switching (ModUp: each digit to the other limbs and the special
 * primes; ModDown: the special primes to the ciphertext limbs) runs fused
 * with the first (column) pass of the forward NTT of its outputs, in
 * workgroups that each own a column tile and a group of outputs; the
 * number of workgroups aimed for (512, 768, 1024 or 1536, which sets the
 * outputs per group) is timed for the top-level ModUp and ModDown and the
 * fastest kept.  target[2] (may be NULL) receives the choice for ModUp and
 * ModDown, us[2][4] (may be NULL) the timings in microseconds. */
int he_ctx_conv_tuning(const he_ctx* ctx, int32_t* target, float* us);
const char* he_last_error(void);

/* Execution lanes.  Calls on different streams of one context may run
 * concurrently on the device: each stream gets its own key-switch workspace
 * and pool of temporary ciphertexts (a "lane", created on first use).  Calls
 * on the same stream are ordered.  he_lane_reserve pre-allocates the lane of
 * `stream` with n_ct_buffers temporaries (so later calls allocate nothing
 * unless a layer needs more); he_lane_release synchronises the stream and
 * frees its lane; he_lane_bytes gives the device bytes of one lane. */
int he_lane_reserve(he_ctx* ctx, he_stream stream, int n_ct_buffers);
int he_lane_release(he_ctx* ctx, he_stream stream);
size_t he_lane_bytes(const he_ctx* ctx, int n_ct_buffers);

/* ------------------------------------------------------------ keys
 * Evaluation keys are the paper's "rotation keys" and relinearization key
 * (Section "Evaluation Keys Management"): preloaded into HBM and kept
 * resident until evicted.  `src` holds one key in the layout above
 * ([dnum][2][L+K][N], host or device memory per src_on_device); the library
 * copies it into its own storage (converted to an internal form).
 * key_id: a rotation amount r (slot i <- slot i + r; ids are reduced mod N/2)
 * or HE_KEY_RELIN.  Uploading over a key that has a device copy first waits
 * for the whole device (work on any stream may still read the old key). */
int he_key_upload(he_ctx* ctx, int32_t key_id, const uint64_t* src, size_t bytes, int src_on_device,
                  he_stream stream);
int he_key_evict(he_ctx* ctx, int32_t key_id);
int he_key_count(const he_ctx* ctx);
size_t he_key_bytes(const he_ctx* ctx); /* bytes of one key */
/* Dynamic key management (section "Evaluation Keys Management": keys loaded
 * on demand and removed at run time, next to preloading).  A key registered
 * with a host copy (copied into library-owned pinned memory; plain limb
 * layout as for he_key_upload) need not be in device memory: any operation
 * that needs it loads it, stream-ordered on that operation's stream
 * (host-to-device copy + conversion), and another stream using it before the
 * load has finished waits for it.  With a device budget (he_key_cache_limit,
 * bytes; 0 = unlimited) a load first evicts the least recently used
 * host-backed keys that no batch holds; an evicted buffer is reused only
 * after the last kernel reading it on every stream that used it has
 * completed (the host waits for that).
 * Keys uploaded with he_key_upload (no host copy) are never evicted; keys a
 * batch captured stay resident until he_batch_destroy.  The budget is soft
 * when nothing is evictable.  he_key_prefetch loads keys ahead of use on the
 * given stream.  he_key_evict drops both copies.  Key-management calls must
 * not run concurrently with other calls on the same context. */
int he_key_host_register(he_ctx* ctx, int32_t key_id, const uint64_t* host_key, size_t bytes);
int he_key_cache_limit(he_ctx* ctx, size_t device_bytes);
int he_key_prefetch(he_ctx* ctx, const int32_t* key_ids, int n, he_stream stream);
/* device bytes of resident keys, loads from host copies and evictions so far */
int he_key_cache_stats(const he_ctx* ctx, size_t* resident_bytes, int64_t* loads, int64_t* evictions);

/* ------------------------------------------------------------ ring ops */
/* In-place negacyclic NTT (inverse = 0) or iNTT (inverse = 1, includes N^-1)
 * of n_limbs consecutive limbs at `poly` ([n_limbs][N], device), limb t taken
 * modulo modulus index first_limb + t.  Moduli indices beyond L-1 address
 * the special primes.  Inputs must be canonical residues (in [0, q)); so are
 * the outputs. */
int he_ntt(he_ctx* ctx, uint64_t* poly, int n_limbs, int first_limb, int inverse, he_stream stream);

/* Slot rotation Rot_r (slot i <- slot i + r), the paper's rotation
 * (Sections "Secure Convolution Layer", Algorithm 1): Galois automorphism
 * X -> X^g, g = 5^(r mod N/2) mod 2N, with hybrid key switching.  Pinned
 * formula: ModUp(c1) -> phi_g on the extended digits -> inner product with
 * evk_r -> ModDown, out = (phi_g(c0) + u0, u1).  Equal to he_rotate_hoisted
 * with one index.  r = 0 (mod N/2) copies.  HE_ENOKEY if evk_r is absent. */
int he_rotate(he_ctx* ctx, const he_ct* in, int32_t r, he_ct* out, he_stream stream);

/* he_rotate for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same rotation, bit for bit, with the key-switch workspace in a static
 * device array of HE_NOALLOC_SCRATCH_BYTES that each GPU the library runs on
 * holds until the process ends, so the call allocates nothing (no lane, no
 * events, no key loads).  The key must be a resident key from he_key_upload
 * (a host-registered key is HE_ENOKEY), profiling must be off, and the key
 * switch at in->level must fit the array: N (l + dnum (l+K) + 2 (l+K) + 2 l)
 * words (l = in->level, dnum = ceil(l / alpha)); larger is HE_EINVAL, with
 * the sizes in he_last_error().  All calls on one GPU share that GPU's
 * array: calls that overlap on one GPU (other streams, other threads, other
 * contexts) race and must be serialised by the caller.  Nothing in the
 * array has to start at zero; it keeps the last call's intermediates. */
#define HE_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int he_rotate_noalloc(he_ctx* ctx, const he_ct* in, int32_t r, he_ct* out, he_stream stream);

/* Hoisted rotations ("fast rotations"): one ModUp of c1 shared by n
 * rotations; outs[t] = Rot_{r[t]}(in).  Outputs must not alias the input or
 * each other (HE_EINVAL); their key switches may run on helper streams of
 * `stream` (he_ctx_layer_streams), all finished in stream order of `stream`.
 * Three or more key switches whose keys are all uploaded (not host-
 * registered) run batched, in rounds of 8: one inner-product launch and one
 * ModDown chain per round (the same residues as key switch by key switch;
 * the stream's lane then holds a round's workspace, 8 x 2 (2L+K) N words). */
int he_rotate_hoisted(he_ctx* ctx, const he_ct* in, const int32_t* r, int n, he_ct* outs, he_stream stream);

/* out (+)= in (.) pt limb-wise at the ciphertext's level (pt-ct product of
 * the paper's convolution/pooling/FC MACs).  accumulate = 0: out = in*pt,
 * out.scale = in.scale * pt.scale.  accumulate = 1: out += in*pt, requiring
 * out.level == in.level and out.scale == in.scale * pt.scale (HE_ESCALE).
 * out may alias in when accumulate == 0. */
int he_mul_plain(he_ctx* ctx, const he_ct* in, const he_pt* pt, he_ct* out, int accumulate, he_stream stream);

/* Sum of plaintext-ciphertext products in one pass (the MAC of the
 * paper's layers, e.g. a kernel vector times each rotated input):
 * out (+)= sum_t cts[t] (.) pts[t], n >= 1 terms at one level whose scale
 * products cts[t].scale * pts[t].scale are all equal (HE_ESCALE); out gets
 * that level and scale.  out must not alias a term. */
int he_mac_plain(he_ctx* ctx, const he_ct* cts, const he_pt* pts, int n, he_ct* out, int accumulate,
                 he_stream stream);

/* Exact ring additions; equal levels (HE_ELEVEL) and equal scales
 * (HE_ESCALE) required.  out may alias a or b. */
int he_add(he_ctx* ctx, const he_ct* a, const he_ct* b, he_ct* out, he_stream stream);
int he_sub(he_ctx* ctx, const he_ct* a, const he_ct* b, he_ct* out, he_stream stream);
/* c0 += pt (scales must match).  out may alias a. */
int he_add_plain(he_ctx* ctx, const he_ct* a, const he_pt* pt, he_ct* out, he_stream stream);

/* Floor rescale by the top prime q_t (t = level-1):
 * c'_i = (c_i - ([c]_{q_t} mod q_i)) q_t^{-1} mod q_i; scale /= q_t.
 * Computed as a ModDown by the single prime q_t (inverse transform of the top
 * limb, its residues reduced to the other limbs in the forward column pass,
 * the combination in the forward row pass).  HE_ELEVEL at level 1.  out may
 * alias in. */
int he_rescale(he_ctx* ctx, const he_ct* in, he_ct* out, he_stream stream);
/* Keep limbs q_0..q_{level-1} (level alignment, no scale change). */
int he_drop_level(he_ctx* ctx, const he_ct* in, int level, he_ct* out, he_stream stream);

/* Ciphertext product with relinearization (no rescale): tensor
 * (a0 b0, a0 b1 + a1 b0, a1 b1), then d2 key-switched with the HE_KEY_RELIN
 * key.  Equal levels required; out.scale = a.scale * b.scale. */
int he_mul_relin(he_ctx* ctx, const he_ct* a, const he_ct* b, he_ct* out, he_stream stream);
/* Relinearize a 3-part ciphertext d ([3][level][N], device) into out. */
int he_relin(he_ctx* ctx, const uint64_t* d, int level, double scale, he_ct* out, he_stream stream);

/* Multiply every slot by i (sign = +1: the monomial X^(N/2), whose slot
 * values zeta^(5^j N/2) are all i) or by -i (sign = -1: -X^(N/2)).  Exact:
 * in NTT form the monomial is +-psi^(N/2) per limb (the sign flips between
 * the two halves of the bit-reversed order); level and scale unchanged.
 * out may alias in. */
int he_mul_i(he_ctx* ctx, const he_ct* in, int sign, he_ct* out, he_stream stream);

/* ModRaise, bootstrapping's first step: limb 0 of `in` (residues mod q_0)
 * read as integers centred in (-q_0/2, q_0/2] (coefficient a in [0, q_0)
 * taken as a - q_0 when a > (q_0 - 1)/2) and reduced modulo q_0..q_{level-1}:
 * inverse transform of limb 0, the lift, forward transform of `level` limbs.
 * The result encrypts m + q_0 I for a small integer polynomial I (|I| at
 * most (h + 1)/2 for a secret of h nonzero ternary coefficients); limb 0 is
 * unchanged, the scale is in.scale.  1 <= level <= L; out must not alias in. */
int he_mod_raise(he_ctx* ctx, const he_ct* in, int level, he_ct* out, he_stream stream);

/* Multiply by a real constant c encoded at `scale` as the constant
 * polynomial llround(c * scale) (ties away from zero); out.scale =
 * in.scale * scale.  Add a real constant c encoded at the ciphertext's own
 * scale.  out may alias in. */
int he_mul_const(he_ctx* ctx, const he_ct* in, double c, double scale, he_ct* out, he_stream stream);
int he_add_const(he_ctx* ctx, const he_ct* in, double c, he_ct* out, he_stream stream);

/* ------------------------------------------------------------ layers
 * Feature-map layout in the slots (the paper's channel-by-channel flattening,
 * Section "Secure Convolution Layer", Fig. "Flattening of an input tensor"):
 * value (c, y, x) sits in slot c*chan_stride + y*row_stride + x for c < C,
 * y < H, x < W; reps = 2 means the C-channel block is stored twice back to
 * back (2*C*chan_stride = N/2 slots), which the special convolution uses to
 * sum input channels by cyclic rotation.  Unused slots hold zeros. */
typedef struct {
  int32_t channels, height, width;
  int32_t row_stride, chan_stride;
  int32_t reps;
} he_fmap;

/* Plan of a layer: the plaintexts it consumes, the distinct rotation keys it
 * needs (the paper's per-layer rotation-index helper, Section "Evaluation
 * Keys Management"), the levels it consumes and the output layout.  rot_keys
 * may be NULL (then only *n_keys is written); otherwise it must hold 64. */
typedef struct {
  int32_t n_kernel_pts, n_mask_pts;
  int32_t n_keys;
  int32_t rot_keys[64];
  int32_t levels;
  int32_t key_switches;
  he_fmap out;
} he_layer_plan;

/* Plaintext recipes (section "FHEON's Support Functions": the model owner
 * preprocesses weights into the plaintext vectors a layer multiplies by).
 * Host only, no context: fills the real slot vectors (N/2 doubles each,
 * N = 2^log_n) a layer consumes, in the order and number its plan gives,
 * for the schedule options in the descriptor (set the same options on the
 * context that runs the layer; the input-channel sum mode does not change
 * the vectors):
 *   HE_LAYER_CONV: weights [out_ch][in.channels][kernel][kernel]; the
 *     plan's n_kernel_pts kernel vectors, then its n_mask_pts masks, then,
 *     when bias (out_ch values) is given, one bias vector (b_f on every
 *     output position of channel f, in every replica of the output layout);
 *   HE_LAYER_AVGPOOL: the n_mask_pts masks (kernel 0 = global pooling);
 *   HE_LAYER_FC: weights [n_out][n_in]; rows form: the n_out rows, then
 *     e_0; diagonal form: the n_in rotated diagonals; then, when bias
 *     (n_out values) is given, the bias in slots 0..n_out-1;
 *   HE_LAYER_CHEB_MASK: he_cheb's scale mask, 1/beta on slots [0, n_in).
 * out: [cap_vectors][N/2] doubles or NULL (then only *n_vectors is set).
 * The caller encodes the vectors (scale and level: kernel vectors at the
 * input's level, masks one level per step lower as the layer consumes them,
 * biases at the output's scale and level).  HE_EINVAL for shapes the layer
 * rejects or a too small cap_vectors; HE_EUNSUPPORTED as the layer. */
#define HE_LAYER_CONV 0
#define HE_LAYER_AVGPOOL 1
#define HE_LAYER_FC 2
#define HE_LAYER_CHEB_MASK 3
typedef struct {
  int32_t kind;
  int32_t log_n;        /* ring degree N = 2^log_n (slots N/2) */
  int32_t mask_chains;  /* HE_CHAIN_HORNER or HE_CHAIN_BSGS (he_ctx_mask_chains) */
  int32_t fc_form;      /* HE_FC_ROWS or HE_FC_DIAG (he_ctx_fc_form) */
  he_fmap in;           /* CONV, AVGPOOL: input layout */
  int32_t out_ch, kernel, stride, padding;
  int32_t n_in, n_out;  /* FC; CHEB_MASK: n_in = used slots */
  double beta;          /* CHEB_MASK */
  int32_t stride_mode;  /* HE_STRIDE_EXTRACT or HE_STRIDE_LOG (he_ctx_striding) */
  int32_t stride_groups; /* HE_STRIDE_JOINT or HE_STRIDE_GROUP_IN (he_ctx_stride_groups) */
  int32_t channel_sum;   /* HE_CHSUM_CHAIN or HE_CHSUM_LOG (he_ctx_conv_channel_sum; keys only) */
} he_layer_desc;
int he_layer_plaintexts(const he_layer_desc* desc, const double* weights, const double* bias, double* out,
                        size_t cap_vectors, int32_t* n_vectors);
/* The layer's plan from its description alone (host only, no context):
 * the distinct rotation keys (the paper's rotation-index helper, which the
 * client uses to generate exactly the keys a model needs), the plaintext
 * counts, levels, key switches and output layout — what he_conv2d_plan,
 * he_avgpool_plan and he_fc_plan give on a context with the same options.
 * CHEB_MASK: one mask plaintext, no keys.  Errors as he_layer_plaintexts. */
int he_layer_rotations(const he_layer_desc* desc, he_layer_plan* plan);

/* Convolution (Sections "Secure Convolution Layer", "Secure Advanced
 * Convolution Layer" with striding approach 1 and the multi-channel striding
 * pipeline, "Special Secure Convolution Layer" with Algorithms 1-3).
 * Supported: kernel 3 / padding 1 on a dense square map that is replicated
 * (reps = 2) or has one channel in and out (special schedule; stride 1 or 2),
 * and every other padding 0 <= P <= (k-1)/2 with any kernel and stride
 * (generic schedule: the zero padding is realised by the kernel vectors, so
 * the output keeps the input's layout).  Larger paddings (section "Secure
 * Advanced Convolution With Padding"): the input is first re-laid out as the
 * padded tensor X_p, (C, H+2P, W+2P) flattened densely (row stride W+2P,
 * channel block (H+2P)(W+2P)), by masked chains over the rows (key
 * rs - (W+2P)) and the channels (key cs - (H+2P)(W+2P)), each only when it
 * moves data (else one clearing mask), and one rotation by -(P (W+2P) + P);
 * the generic schedule with P = 0 then runs on X_p.  C (H+2P)(W+2P) must fit
 * the slots; a layer needing more than 64 rotation keys: HE_EUNSUPPORTED.
 * Plaintexts (NTT form, at least the input level in limbs, encoded at one
 * common scale), in this order:
 *  special: kernel_pts[9 f + t], t = 3 (dy+1) + (dx+1): K[f, b mod C, t] on
 *    block b of every replica, times the Algorithm-3 mask of tap t;
 *    mask_pts: F block masks (1 on block f of every output replica) when
 *    C > 1 or F > 1, then the stride-compaction masks.
 *  generic: kernel_pts[k*k f + i k + j]: K[f, c, i, j] at c*cs + y*rs + x for
 *    the stride-1 outputs (y < H+2P-k+1, x < W+2P-k+1) whose neighbour
 *    (y+i-P, x+j-P) lies inside the image, 0 elsewhere (tap (i, j) is the
 *    input rotated by (i-P) rs + (j-P)); mask_pts: the block-0 mask of the
 *    stride-1 outputs when C > 1, then the stride-compaction masks.
 *  compaction masks (stride S > 1, outputs (S i, S j) -> dense Ho x Wo):
 *    Wo column masks (1 at c*cs + S i rs + S j, all c, i), Ho row masks
 *    (1 at c*cs + S i rs + j, j < Wo), then C channel masks (1 on
 *    c*cs + [0, Ho*Wo)) — each step only when it moves data.
 *  padded (P > (k-1)/2): kernel_pts as generic for X_p with P = 0; mask_pts:
 *    first the re-layout masks at the input level (channel step: C masks,
 *    1 on channel c's image; row step: H masks, 1 on row y of every
 *    channel; each on the layout its step sees, in the step order of the
 *    plan; or the one clearing mask of the whole image), then the generic
 *    masks for X_p.
 * The result is rescaled after every multiplicative level. */
int he_conv2d_plan(const he_ctx* ctx, const he_fmap* in_map, int out_ch, int kernel, int stride, int padding,
                   he_layer_plan* plan);
/* Input-channel sum of he_conv2d (S = sum_{j < C} Rot_{j step}(A), step =
 * W^2 for the special schedule, chan_stride for the generic one), chosen per
 * context for plans and calls made after this call:
 *   HE_CHSUM_CHAIN (default): the paper's chain with the single key step
 *     (Algorithm 1 of "Special Secure Convolution Layer"), C - 1 key switches
 *     per output channel;
 *   HE_CHSUM_LOG: for C a power of two, doubling S <- S + Rot_{2^t step}(S),
 *     t < log2 C: log2 C key switches per output channel and log2 C keys
 *     (2^t step); other channel counts keep the chain.
 * Both give the same plaintext; the ciphertexts differ (other keys, other
 * key-switch noise).  HE_EINVAL for another mode. */
#define HE_CHSUM_CHAIN 0
#define HE_CHSUM_LOG 1
int he_ctx_conv_channel_sum(he_ctx* ctx, int mode);
/* Masked rotation chains sum_{t<n} Rot_{t key}(v . m_t) of the layers (the
 * three stride-compaction steps of he_conv2d / he_avgpool and the channel
 * gather of global pooling), chosen per context for later plans and calls:
 *   HE_CHAIN_HORNER (default): acc = RS(v.m_{n-1}); acc = Rot_key(acc) +
 *     RS(v.m_t), n - 1 key switches, one key;
 *   HE_CHAIN_BSGS: baby-step giant-step with B = ceil(sqrt n), A =
 *     ceil(n / B): one hoisted group of the rotations b key (b < B) of v, inner
 *     sums I_a = RS(sum_b Rot_{b key}(v) . m_{aB+b}) and a Horner chain over a
 *     with key B key: (B - 1) + (A - 1) key switches, B keys.  The caller
 *     supplies mask t = a B + b rotated by b key (Rot_{b key}(m_t)), in the
 *     same order and number as for Horner.
 * Same plaintext result, other ciphertexts.  HE_EINVAL for another mode. */
#define HE_CHAIN_HORNER 0
#define HE_CHAIN_BSGS 1
int he_ctx_mask_chains(he_ctx* ctx, int mode);
/* Column step of the stride compaction (section "Secure Advanced Convolution
 * With Striding"), chosen per context for later plans and calls:
 *   HE_STRIDE_EXTRACT (default, the paper's first approach): one masked
 *     chain over the Wo columns with key S-1 (Wo - 1 key switches, 1 level);
 *   HE_STRIDE_LOG (its second approach): ceil(log2 Wo) steps t, each a
 *     two-term masked chain with key (S-1) 2^t that keeps the columns j
 *     whose bit t is 0 and moves those whose bit t is 1 left by (S-1) 2^t
 *     (one key switch and one level per step): fewer rotations and keys
 *     (log2 Wo + 1 for one channel), more levels.  Step t's masks: mask 0
 *     is 1 (the column scale at t = 0) at c*cs + S i rs + S (j - j mod 2^t)
 *     + j mod 2^t for the j with bit t clear, mask 1 the same for bit t set;
 *     Wo = 1 keeps the one-mask column step.
 * The row and channel steps are the same in both.  Same plaintext result.
 * HE_EINVAL for another mode. */
#define HE_STRIDE_EXTRACT 0
#define HE_STRIDE_LOG 1
int he_ctx_striding(he_ctx* ctx, int mode);
/* Output-channel grouping of a strided convolution's compaction (section
 * "Secure Advanced Convolution With Striding", the multi-channel pipeline),
 * per context for later plans and calls:
 *   HE_STRIDE_JOINT (default): all F output channels compacted at once;
 *   HE_STRIDE_GROUP_IN: the paper's groups of g = the layer's input channels
 *     (when fewer than F): each group compacted jointly (its masks in the
 *     group order, covering only its channels; a one-channel group keeps the
 *     channel step as one mask), then the groups merged by a Horner chain
 *     with the single key g (cs - Ho Wo), G - 1 more key switches, no level.
 * Same plaintext result.  HE_EINVAL for another mode. */
#define HE_STRIDE_JOINT 0
#define HE_STRIDE_GROUP_IN 1
int he_ctx_stride_groups(he_ctx* ctx, int mode);
/* bias_pt (nullable): the output channels' biases on the output layout
 * (he_layer_plaintexts), encoded at the output's scale and level, added to
 * the result (the convolution's "add the bias"). */
int he_conv2d(he_ctx* ctx, const he_ct* in, const he_fmap* in_map, int out_ch, int kernel, int stride, int padding,
              const he_pt* kernel_pts, int n_kernel_pts, const he_pt* mask_pts, int n_mask_pts, const he_pt* bias_pt,
              he_ct* out, he_fmap* out_map, he_stream stream);

/* Average pooling (Section "Secure Average Pooling Layer", equation of the
 * pooled output): window sum by rotations, 1/k^2 folded into the column masks
 * of the stride compaction (stride 1: one mask of 1/k^2 on the valid
 * outputs).  kernel = 0 selects global average pooling: per-channel sums by
 * log-step rotations, then channel c gathered into slot c with masks of
 * 1/(H W) at slot c*cs (requires dense power-of-two channel blocks). */
int he_avgpool_plan(const he_ctx* ctx, const he_fmap* in_map, int kernel, int stride, he_layer_plan* plan);
int he_avgpool(he_ctx* ctx, const he_ct* in, const he_fmap* in_map, int kernel, int stride, const he_pt* mask_pts,
               int n_mask_pts, he_ct* out, he_fmap* out_map, he_stream stream);

/* Fully connected y = W x (+ b) (Section "Secure Fully Connected Layer"):
 * input in slots 0..n_in-1 (n_in a power of two); weight_pts[k] holds row
 * W_k in slots 0..n_in-1; mask_pts[0] is e_0 (1 in slot 0).  Each neuron is
 * a product, a log-step sum into slot 0 and an e_0 mask; the outputs are
 * merged into slots 0..n_out-1 with the single key -1.  bias_pt (nullable)
 * must carry the output scale. */
int he_fc_plan(const he_ctx* ctx, int n_in, int n_out, he_layer_plan* plan);
int he_fc(he_ctx* ctx, const he_ct* in, int n_in, int n_out, const he_pt* weight_pts, const he_pt* mask_pts,
          const he_pt* bias_pt, he_ct* out, he_stream stream);
/* Form of later he_fc plans and calls:
 *   HE_FC_ROWS (default): the per-neuron schedule above, n_out products,
 *     n_out log2(n_in) + n_out - 1 key switches, two levels;
 *   HE_FC_DIAG: the diagonal (Halevi-Shoup) form for n_out <= n_in with
 *     baby-step giant-step (B = ceil(sqrt n_in), A = n_in / B rounded up):
 *     x~ = x + Rot_{-n_in}(x), one hoisted group Rot_b(x~) (b < B), inner
 *     sums I_a = sum_b Rot_b(x~) . w_{aB+b}, acc = I_{A-1}; acc = Rot_B(acc)
 *     + I_a, one rescale: 1 + (B - 1) + (A - 1) key switches, one level.
 *     weight_pts[d] (d < n_in) is diagonal d, W[j][(j + d) mod n_in] in slot
 *     j < n_out, rotated by -(d / B) B; no mask_pts.  The input must be zero
 *     in slots [n_in, 2 n_in) and in the top n_in slots (as global pooling
 *     leaves it); the output is zero outside slots 0..n_out-1.
 * HE_EINVAL for another mode. */
#define HE_FC_ROWS 0
#define HE_FC_DIAG 1
int he_ctx_fc_form(he_ctx* ctx, int mode);

/* Streams the independent parts of a call are spread over (1..8, default 2):
 * the per-channel work (products with the kernel vectors, input-channel sum,
 * masking) of a convolution's output channel f, the per-neuron work of the
 * per-row fully connected form (product, log-step sum, mask), the products
 * of he_cheb (on two streams at most: its Chebyshev terms by list scheduling
 * and the remainder branch of its division tree), and key switch j (inner
 * product + ModDown after the shared ModUp) of a hoisted rotation set with
 * several keys, run on the caller's stream (index mod n == 0) or on helper
 * stream (index mod n) of the caller's stream, which the library creates on
 * first use (default priority, one workspace lane each: he_lane_bytes(0) of
 * device memory per helper) and destroys with he_lane_release of the
 * caller's stream or with the context.  The helpers start after the work
 * already enqueued on the caller's stream, and the caller's stream waits for
 * them before the parts are combined (or the call returns), so the call stays
 * stream-ordered on the caller's stream and its results are the same for
 * every n.  Rings below N = 2^16 always use the caller's stream alone (their
 * key switches are too short to cover the cross-queue waits).  The gain needs
 * the helpers on other hardware queues than the caller's (HIP maps streams
 * onto a few queues per process).  HE_EINVAL outside [1, 8]. */
int he_ctx_layer_streams(he_ctx* ctx, int n);

/* Polynomial activation p(x) = c[0] + c[1] x + c[2] x^2 + c[4] x^4 (c[3]
 * must be 0) in three levels with two relinearizations:
 * x2 = RS(x*x); t = RS(x2 * c4 @delta) + c2; v = RS(x2 * t);
 * lin = RS(x * c1 @sigma) with sigma = s_v q / s_x so lin lands on v's level
 * (its scale is set to s_v); p = v + lin + c0.  With c = the least-squares
 * fit of max(0, x) on [-1, 1] this is the LeNet-5-shaped stack's ReLU. */
int he_poly4(he_ctx* ctx, const he_ct* in, const double* c, double delta, he_ct* out, he_stream stream);

/* Secure ReLU by Chebyshev interpolation (section "Activation Function
 * (Secure ReLU)" and its algorithm): with a scale mask (1/beta on the n used
 * slots, encoded by the caller at scale delta; NULL when beta <= 1) the
 * input is first multiplied by it and rescaled; then
 *   y = c_0 / 2 + sum_{j=1..degree} c_j T_j(v)
 * is evaluated by baby-step giant-step division: the series is split
 * recursively as q T_K + r by giant steps T_K (K = 8 * 2^m, the largest not
 * above the degree of the part being split; T_{K+i} = 2 T_K T_i - T_{K-i})
 * down to leaves of degree below 8.  The T_j needed (leaf terms with nonzero
 * coefficients, T_1, the giant steps and their factors) are built by
 * T_{2k} = 2 T_k^2 - 1, T_{2k+1} = 2 T_k T_{k+1} - T_1, each product
 * relinearized and rescaled.  Each subtree is evaluated onto a target level
 * and scale: a leaf as sum c_j T_j, each term by a constant multiplication
 * encoded at target * q / scale(T_j), plus its constant; a node as
 * RS(Relin(q' T_K)) + r' with q' evaluated one level higher.  Degree 59 with
 * a mask: 14 relinearizations, 7 levels.  Levels consumed and
 * relinearizations: he_cheb_plan.  out
 * gets level in->level - levels, scale delta.  HE_ELEVEL without enough
 * levels, HE_ENOKEY without the relinearization key, HE_EINVAL for a degree
 * outside [1, HE_CHEB_MAX_DEGREE] or when every c_j (j >= 1) is zero. */
#define HE_CHEB_MAX_DEGREE 255
int he_cheb(he_ctx* ctx, const he_ct* in, const he_pt* scale_mask, const double* coeffs, int degree, double delta,
            he_ct* out, he_stream stream);
/* Levels consumed and relinearizations of he_cheb for these coefficients
 * (host only). */
int he_cheb_plan(const double* coeffs, int degree, int masked, int32_t* levels, int32_t* relins);
/* Coefficients c_0..c_degree of the Chebyshev interpolant of
 * f(z) = beta max(0, z) on [-1, 1] at the degree + 1 first-kind nodes
 * cos(pi (k + 1/2) / (degree + 1)) (f ~ c_0 / 2 + sum c_j T_j); c_1 = beta/2
 * and the other odd coefficients are exactly 0.  The paper's default
 * degree is 59.  Host only; `coeffs` holds degree + 1 doubles. */
int he_cheb_relu_coeffs(double beta, int degree, double* coeffs);

/* ------------------------------------------------------------ bootstrapping
 * The paper's bootstrapping support function (Section "FHEON's Support
 * Functions"; its deep models refresh ciphertexts between layers), which it
 * takes from its CPU library without describing it.  Here the standard
 * four stages, each a composition of the calls above:
 *  1. ModRaise (he_mod_raise) of limb 0 to level `level` (0: L); the result,
 *     t = m + q_0 I, is relabelled 2^e delta with e the smallest integer such
 *     that 2^e delta >= 2 q_0 k_min (k_min bounds |I| + 1/2); the EvalMod
 *     range is then K = 2^e delta / (2 q_0).
 *  2. CoeffToSlot: the inverse of the slot decoding map (evaluation at
 *     zeta^(5^j)) as log2(N/2) radix-2 butterfly stages, h = N/4 .. 1,
 *     grouped into `levels` levels (as even as possible, larger first).
 *     Each level is a sum of diagonals D_d (.) Rot_d(x) evaluated baby-step
 *     giant-step: the shifts are multiples of the level's smallest stage u,
 *     d = u k with k centred modulo N/(2u), k = i + B j with B the smallest
 *     power of two with B^2 >= kmax - kmin + 1; baby rotations Rot_{u i}
 *     (one hoisted set), for each giant j ascending
 *     s_j = RS(sum_i pt_{j,i} (.) Rot_{u i}(x)), rotated by u B j when j != 0,
 *     summed.  pt_{j,i} holds D_{u(i+Bj)} rotated by -u B j.  The output
 *     holds (t_lo + i t_hi) / (2 q_0 K) in bit-reversed slot order.
 *  3. EvalMod: w = conj(x) (HE_KEY_CONJ); re = x + w; im = -i (x - w);
 *     each through he_cheb (no mask, output scale delta) with the Chebyshev
 *     interpolant of he_boot_mod_coeffs: with r = double_angles = 0 the
 *     sine sin(2 pi K x) / (2 pi) directly; with r > 0 the cosine
 *     cos(2 pi (K x - 1/4) / 2^r), then r double angles
 *     p = RS(Relin(c c)), c = (p + p) - 1 (ending at sin(2 pi K x)) and the
 *     scale label times 2 pi.  Either removes q_0 I and leaves about
 *     m / q_0; z = re + i im.
 *  4. SlotToCoeff: the forward stages h = 1 .. N/4 (CoeffToSlot's groups
 *     mirrored), same evaluation; the result is relabelled
 *     scale(z) * in.scale / q_0 and decrypts to the input's message.
 * Plaintext scales: CoeffToSlot level g (at level - g) encodes its
 * plaintexts at q 2^-e_g, SlotToCoeff level g (at its level l) at
 * q 2^f_g, q the prime that level's rescale removes; e_g split e and f_g
 * split round(log2(q_0 / (delta a))) (a = 2 pi with double angles, else 1)
 * as evenly as possible, larger first (he_boot_scales).  Levels consumed:
 * 2 * levels + he_cheb_plan's count + r.  The client's secret should be
 * sparse (Hamming weight h) so that |I| <= (h + 1) / 2 stays below k_min:
 * a multiple of q_0 outside [-K, K] is not removed.
 * Key switches: the transforms' rotations (he_boot_plan), one
 * conjugation and he_cheb's relinearizations twice.  The giant steps of each
 * transform level (round-robin, each stream keeping a partial sum) and the
 * two EvalMod parts run on up to he_ctx_layer_streams streams at every ring
 * degree (at N = 2^16, where he_cheb forks a helper of its own stream, the
 * second part runs on the caller's second helper stream, so the parts
 * overlap); the result does not depend on the split. */
typedef struct {
  int32_t levels;        /* levels per linear transform, 1..log2(N/2) */
  int32_t degree;        /* EvalMod Chebyshev degree, 1..HE_CHEB_MAX_DEGREE */
  int32_t level;         /* ModRaise target level (0: L) */
  int32_t double_angles; /* r, 0..8 (0: the sine directly) */
  double k_min;          /* bound on |I| + 1/2 */
  double delta;          /* EvalMod input (Chebyshev output) scale */
} he_boot_desc;

#define HE_BOOT_MAX_ROTATIONS 256
/* Plan of the two linear transforms for N = 2^log_n and `levels` levels
 * (host only): the distinct rotation amounts (in [1, N/2), ascending) both
 * transforms use, the plaintext count of each level in application order
 * (CoeffToSlot then SlotToCoeff, `levels` each) and the key switches both
 * transforms perform (baby steps plus nonzero giant steps; may be NULL).
 * rotations holds HE_BOOT_MAX_ROTATIONS entries, counts 2 * levels. */
int he_boot_plan(int32_t log_n, int32_t levels, int32_t* rotations, int32_t* n_rotations, int32_t* counts,
                 int32_t* n_key_switches);
/* The plaintext slot vectors (complex, N/2 slots each, real parts in re,
 * imaginary parts in im) of one transform (inverse = 1: CoeffToSlot, 0:
 * SlotToCoeff) in consumption order: level by level, giant j ascending,
 * baby i ascending (pt_{j,i} above).  Pure butterfly products (no scale
 * constant); `cap` = doubles available in each of re, im (host only). */
int he_boot_diagonals(int32_t log_n, int32_t levels, int32_t inverse, double* re, double* im, size_t cap);
/* Chebyshev coefficients c_0..c_degree, interpolated on [-1, 1] at the
 * degree + 1 first-kind nodes, of sin(2 pi K x) / (2 pi) (double_angles = 0;
 * even coefficients exactly 0) or cos(2 pi (K x - 1/4) / 2^double_angles). */
int he_boot_mod_coeffs(double K, int32_t degree, int32_t double_angles, double* coeffs);
/* For a context and description: the EvalMod range K, the raise label
 * 2^e delta, and the plaintext scales of every CoeffToSlot and SlotToCoeff
 * level (`levels` doubles each) at the levels the procedure uses them. */
int he_boot_scales(const he_ctx* ctx, const he_boot_desc* desc, double* K, double* raise_scale, double* cts_scales,
                   double* stc_scales);
/* Refresh `in` (any level; limb 0 is used).  cts_pts, stc_pts: the
 * plaintexts of he_boot_diagonals encoded at he_boot_scales (level g of
 * CoeffToSlot at level - g, SlotToCoeff level g at the level it is applied
 * at); coeffs: he_boot_mod_coeffs(K, degree, double_angles).  Needs the
 * rotation keys of he_boot_plan, HE_KEY_CONJ and HE_KEY_RELIN.  out gets
 * level level - 2 levels - he_cheb_plan levels - double_angles.  HE_ELEVEL
 * when the chain is too short, HE_ENOKEY for a missing key. */
int he_bootstrap(he_ctx* ctx, const he_ct* in, const he_boot_desc* desc, const he_pt* cts_pts, const he_pt* stc_pts,
                 const double* coeffs, he_ct* out, he_stream stream);

/* ------------------------------------------------------------ graph capture
 * Record a sequence of library calls issued on `stream` (a layer schedule,
 * a chain of layers, a bootstrap) into a hipGraph once and replay it as one
 * launch.  Between he_capture_begin and he_capture_end the calls are
 * recorded, not run (relaxed capture mode); the helper streams a call forks
 * join back inside the capture.  The graph keeps the buffers the calls
 * used: inputs, outputs, plaintexts and keys by address, and the stream's
 * own temporaries, so a replay reads whatever those inputs hold then and
 * writes the same outputs.  Rules: run the same sequence once eagerly on the
 * stream first (that allocates the lane, helper streams and temporaries the
 * calls need, which a capture must not); keys must be resident (uploaded
 * with he_key_upload; a key with a host copy fails with HE_EUNSUPPORTED
 * during capture); profiling must be off; replay on the capture stream
 * (its temporaries belong to that stream's lane); keep every captured buffer
 * and key alive while the graph exists.  The stream must not be the null
 * stream.  he_bootstrap at N >= 2^16 refuses to be captured
 * (HE_EUNSUPPORTED): its capture is verified at N = 2^12 only. */
typedef struct he_graph he_graph;
int he_capture_begin(he_ctx* ctx, he_stream stream);
int he_capture_end(he_ctx* ctx, he_stream stream, he_graph** out);
int he_graph_launch(he_graph* graph, he_stream stream);
int he_graph_destroy(he_graph* graph);

/* ------------------------------------------------------------ batching
 * Many ciphertexts, each with its own hoisted rotation set and its own
 * number of outputs:
 *   out[i, o] = RS( sum_t pool[pt_index(i, o, t)] (.) Rot_{rots_i[t]}(in_i) )
 * (the multiply-accumulate of rotated copies that every convolution and
 * pooling stage of the paper's layers performs, Section "Secure Convolution
 * Layer").  All inputs share one level l >= 2 and scale; the result has
 * level l-1 and scale in_scale * pt_scale / q_{l-1}, and is bit-identical to
 * he_rotate_hoisted + he_mul_plain (accumulate) + he_rescale per output.
 * Layouts (device memory, caller-owned, kept alive while the batch exists):
 *   in      [n_items][2][l][N]
 *   pool    [n_pool][pool_level][N] (pool_level >= l)
 *   out     [sum n_out][2][l-1][N], item-major, outputs in order
 * Host arrays (copied at creation): n_rot[i] (1..64 distinct non-zero
 * amounts per item, keys resident), rots (concatenated), n_out[i] >= 1,
 * pt_index (for item i: n_out[i] x n_rot[i] pool indices, o-major).
 * The batched schedule runs ModUp once per input, one key inner product per
 * distinct key for all its ciphertexts, batched ModDown, one fused
 * multiply-accumulate kernel and chunked rescaling.  HE_BATCH_GRAPH: the
 * first he_batch_run on a (non-default) stream captures the schedule in a
 * hipGraph, later runs replay it.  The fused multiply-accumulate keeps a
 * group of outputs in registers and reads an item's rotated copies once per
 * group: variants (outputs per group, polynomials per workgroup) = (4, 2),
 * (8, 2), (16, 2) (the default), (16, 1), (32, 1); HE_BATCH_MAC4 takes
 * (4, 2), HE_BATCH_MAC_SELECT(v) variant v (and skips the tuning);
 * HE_BATCH_TUNE times every variant on the batch's own shapes at creation
 * and keeps the fastest.  All variants give the same bits.  Workspace memory is allocated at creation
 * and released by he_batch_destroy. */
#define HE_BATCH_GRAPH 1
#define HE_BATCH_MAC4 2
#define HE_BATCH_TUNE 4
#define HE_BATCH_MAC_SELECT(v) (((v) + 1) << 8)
typedef struct he_batch he_batch;
typedef struct {
  int32_t n_items;
  int32_t level;
  double in_scale, pt_scale;
  const uint64_t* in;
  const int32_t* n_rot;
  const int32_t* rots;
  const int32_t* n_out;
  const uint64_t* pool;
  int32_t n_pool, pool_level;
  const int32_t* pt_index;
  uint64_t* out;
} he_batch_desc;
int he_batch_create(he_ctx* ctx, const he_batch_desc* desc, int flags, he_batch** out);
int he_batch_run(he_batch* batch, he_stream stream);
/* The same work through the per-op entry points, one ciphertext at a time
 * (the plain path the batched schedule is measured against). */
int he_batch_run_plain(he_batch* batch, he_stream stream);
int he_batch_info(const he_batch* batch, int32_t* total_rotations, int32_t* total_outputs, int32_t* distinct_keys,
                  double* out_scale);
/* The MAC variant in use (outputs per register group, polynomials per
 * workgroup) and, after HE_BATCH_TUNE, the timed milliseconds of every
 * variant in the order above (0 when not tuned); ms (nullable) needs cap >=
 * HE_BATCH_MAC_VARIANTS entries, else HE_EINVAL. */
#define HE_BATCH_MAC_VARIANTS 5
int he_batch_tuning(const he_batch* batch, int32_t* outputs_per_group, int32_t* polys_per_group, float* ms,
                    int32_t cap);
int he_batch_destroy(he_batch* batch);

/* ------------------------------------------------------------ measurement
 * Per-kernel timing: after he_profile_begin, every kernel launch of this
 * context is bracketed by a HIP event pair on its stream.  he_profile_end
 * synchronises those events and writes a JSON object
 *   {"<kernel>": {"launches": n, "ms": total, "bytes": B, "modmul": M}, ...}
 * to `out` (B = algorithmic HBM bytes the launches must move, M = modular
 * products they compute), returning its length or HE_EINVAL if cap is too
 * small.  Profiling adds an event record per launch; leave it off when timing
 * end-to-end throughput. */
int he_profile_begin(he_ctx* ctx);
int he_profile_end(he_ctx* ctx, char* out, size_t cap);

#ifdef __cplusplus
}
#endif
#endif /* HE_H_ */
