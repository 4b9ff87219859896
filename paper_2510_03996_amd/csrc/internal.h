// Library-internal context, tables and helpers (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/he.h"
#include "elem_core.h"

namespace he {

constexpr int MAXL = 64;  // max limbs in any basis (L + K)
constexpr int NTT_VARIANTS = HE_NTT_VARIANTS;  // (tile, residues per thread) kernel shapes

// Basis-conversion tables of one level: device descriptors (one per digit
// for ModUp, one for ModDown) plus the largest output, part and input counts.
struct ConvSet {
  ConvDesc* d = nullptr;  // device array
  int count = 0;
  int max_out = 0;
  int max_parts = 0;
  int max_in = 0;
  std::vector<int> nout, nint;  // per descriptor (host copies)
};

// Optional per-kernel timing: a HIP event pair around each launch on its own
// stream, plus the algorithmic bytes and modular products that launch moves.
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
  double bytes, modmul;
  double ideal_s;  // the launch's modular products at the ALU peak of their arithmetic
};

// ALU peaks of one modular product, from the unit counts (256 CUs x 4 SIMDs
// x 16 lanes at 2.4 GHz = 39.3e12 full-rate lane operations per second):
// an integer Shoup product (64-bit primes) is 10 32-bit multiplies, which
// issue at half rate; a centred FP64 product (primes below 2^50) is 6 FP64
// operations (mul, rint, mul, fma, fma, add), all full rate.
constexpr double LANE_OPS_PER_S = 256.0 * 4 * 16 * 2.4e9;
constexpr double PEAK_MODMUL_INT = LANE_OPS_PER_S / 2 / 10;  // 1.966e12 / s
constexpr double PEAK_MODMUL_F64 = LANE_OPS_PER_S / 6;       // 6.554e12 / s

// One evaluation key.  A key with a host copy may be evicted from device
// memory (its buffer is reused only after the event recorded at its last use
// has completed) and is loaded again, stream-ordered, by the next operation
// that needs it; a key without one stays resident until he_key_evict.
struct KeyEntry {
  uint64_t* dev = nullptr;         // device copy, Montgomery form
  uint64_t* host = nullptr;        // pinned host copy, plain form (library-owned)
  // per stream: recorded after the last kernel on that stream that read dev
  // (host-backed keys only: they are the ones that can be evicted)
  std::vector<std::pair<hipStream_t, hipEvent_t>> uses;
  hipEvent_t ready = nullptr;      // recorded after the last load into dev
  hipStream_t ready_stream = nullptr;
  uint64_t tick = 0;               // LRU clock of the last acquire
  int locks = 0;                   // batches that captured dev
};

// Per-stream execution lane: the key-switch workspace and the pool of
// temporary ciphertext buffers used by work enqueued on one stream.  Work on
// different streams never shares scratch memory, so requests issued on
// different streams may overlap on the device.
// Per-launch tables of the batched hoisted key switch (he_rotate_hoisted with
// several key switches): the key and Galois element of each rotation and the
// two output polynomials of each.  Written on the lane's stream by a one-thread
// kernel before the launches that read it (stream order keeps it stable).
constexpr int SET_MAX = 8;
constexpr int HOIST_SET_MIN = 2;  // key switches from which a hoisted set is batched
struct SetTab {
  const uint64_t* key[SET_MAX];
  uint32_t g[SET_MAX];
  uint32_t ginv[SET_MAX];  // g^-1 mod 2N (the inner product's source-block order)
  uint64_t* out[2 * SET_MAX];
};

struct Lane {
  uint64_t* ws = nullptr;
  std::vector<uint64_t*> ct_pool;  // free [2][L][N] buffers
  std::vector<uint64_t*> ct_all;   // every buffer this lane allocated
  // batched hoisted key switch: SET_MAX x ([2][L+K][N] u + [2][L][N] y) and
  // its table, allocated on first use
  uint64_t* set_ws = nullptr;
  SetTab* set_tab = nullptr;
};

struct Ctx {
  int device = 0;
  int log_n = 0, n = 0, L = 0, K = 0, alpha = 0;
  std::vector<uint64_t> mod;  // L + K moduli
  std::vector<uint64_t> psi;
  std::vector<ModInfo> hmod;
  ModInfo* d_mod = nullptr;
  uint64_t *d_tw = nullptr, *d_twp = nullptr, *d_itw = nullptr, *d_itwp = nullptr;  // [L+K][N]
  // FP64 twiddles w and w/q (used for primes below 2^50)
  double *d_dtw = nullptr, *d_dtwq = nullptr, *d_ditw = nullptr, *d_ditwq = nullptr;
  // modup[level][digit]; moddown[level]
  std::vector<ConvSet> modup, moddown;
  std::vector<ConvSet> rsconv;  // rescale at level l: q_{l-1} -> q_0..q_{l-2} (l >= 2)
  // per level: [L+K][4] finishing constants of the inverse transforms that
  // feed the conversions (conv_fin_fill): N^{-1} (Qin/q_m)^{-1} mod q_m
  std::vector<uint64_t*> d_fin;
  std::vector<LimbMap> modup_ntt;  // per level: every converted limb of every digit (ext-relative)
  // per level l (>= 2): q_{l-1}^{-1} mod q_i (i < l-1) as [l-1] integers, [l-1]
  // Shoup companions, then (double bits) [l-1] values and [l-1] values / q_i:
  // the layout of NttEpi::pinv, so the rescale reuses the ModDown epilogue
  std::vector<uint64_t*> d_rescale;
  // per level l: Shoup pairs of P^{-1} mod q_i: [2][l]
  std::vector<uint64_t*> d_pinv;
  // evaluation keys by normalised id: device copy (Montgomery form) and/or a
  // pinned host copy from which the key is loaded on demand
  std::map<int32_t, KeyEntry> keys;
  std::vector<uint64_t*> key_free;  // device buffers of evicted keys, reused
  size_t key_limit = 0;             // device bytes for keys (0: unlimited)
  uint64_t key_tick = 0;            // LRU clock
  long long key_loads = 0, key_evictions = 0;
  size_t key_words = 0;
  // workspace pool (one key switch at the top level)
  uint64_t* ws = nullptr;
  size_t ws_words = 0;
  std::vector<void*> allocs;
  // execution lanes by stream (the default stream's lane uses `ws`)
  std::map<hipStream_t, Lane*> lanes;
  std::mutex lanes_mu;
  bool prof_on = false;
  size_t lds_per_block = 65536;  // device limit on a workgroup's LDS (bytes)
  int chsum = HE_CHSUM_CHAIN;      // convolution input-channel sum (he_ctx_conv_channel_sum)
  int chain = HE_CHAIN_HORNER;     // masked rotation chains of the layers (he_ctx_mask_chains)
  int stride = HE_STRIDE_EXTRACT;  // column step of the stride compaction (he_ctx_striding)
  int stride_groups = HE_STRIDE_JOINT;  // output-channel groups of a convolution's striding (he_ctx_stride_groups)
  int fc = HE_FC_ROWS;             // fully connected form (he_ctx_fc_form)
  int layer_streams = 2;           // streams a convolution / hoisted set is spread over (he_ctx_layer_streams)
  // helper streams only where a key switch outlasts the fork and join even
  // when the helpers sit on other hardware queues (N = 2^16)
  int streams_for_ring() const { return n >= 65536 ? layer_streams : 1; }
  // helper streams of each caller stream (created on first use, default
  // priority; each gets its own lane), guarded by lanes_mu
  std::map<hipStream_t, std::vector<hipStream_t>> aux_streams;
  // NTT variant (log2 residues per thread) per batch-size bucket (<= 8, 16,
  // 32, more limbs), chosen by the autotuner at context creation
  int ntt_var[4] = {0, 0, 0, 2};           // NTT variant per batch-size bucket
  int conv_target[2] = {1024, 1024};       // conversion workgroup target: ModUp, ModDown (conv_autotune)
  float conv_tune_us[2][4] = {};           // [ModUp / ModDown][candidate] timed microseconds
  float ntt_tune_us[NTT_VARIANTS][4] = {};  // [variant][probe 8/16/32/64 limbs] forward+inverse us
  std::vector<ProfRec> prof;

  int dnum(int level) const { return (level + alpha - 1) / alpha; }
  size_t limb_words() const { return (size_t)n; }
};

// RAII timing scope around one kernel launch (no-op unless profiling is on)
struct ProfScope {
  Ctx* c;
  hipStream_t s;
  ProfRec r;
  bool on;
  // ideal_s < 0: every product priced as an integer Shoup product
  ProfScope(Ctx* c_, const char* name, hipStream_t s_, double bytes, double modmul, double ideal_s = -1.0)
      : c(c_), s(s_), on(c_->prof_on) {
    if (!on) return;
    r.name = name;
    r.bytes = bytes;
    r.modmul = modmul;
    r.ideal_s = ideal_s >= 0.0 ? ideal_s : modmul / PEAK_MODMUL_INT;
    hipEventCreate(&r.a);
    hipEventCreate(&r.b);
    hipEventRecord(r.a, s);
  }
  ~ProfScope() {
    if (!on) return;
    hipEventRecord(r.b, s);
    c->prof.push_back(r);
  }
};

// thread-local error reporting
int set_error(int code, const std::string& msg);
int hip_error(hipError_t e, const char* what);
#define HE_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_error(e_, #call); \
  } while (0)

// NTT over the limbs listed in `map`, for nbatch arrays batch_stride words
// apart (all arrays share the map).
int ntt_launch(Ctx* c, uint64_t* data, size_t batch_stride, int nbatch, const LimbMap& map, bool inverse,
               hipStream_t s);
// out-of-place: the first pass reads from `src` (same positions, batch stride
// src_bs), later passes work on `data`
int ntt_launch_strided(Ctx* c, const uint64_t* src, size_t src_bs, uint64_t* data, size_t batch_stride, int nbatch,
                       const LimbMap& map, bool inverse, hipStream_t s);
int ntt_launch_from(Ctx* c, const uint64_t* src, uint64_t* data, size_t batch_stride, int nbatch, const LimbMap& map,
                    bool inverse, hipStream_t s);
LimbMap range_map(int first_pos, int n, int first_mod);
int ntt_autotune(Ctx* c);
// ModDown epilogue fused into the last forward NTT pass: the transform's
// output y never reaches HBM; instead, for z = 0, 1 and every q-limb i,
//   out_z[i][k] = add_z[i][src_z(k)] + (u_z[i][k] - y_z[i][k]) P^{-1} mod q_i
// with src_0 the automorphism phi_g (g = 1: identity), src_1 the identity;
// a null add_z counts as zero.
struct NttEpi {
  const uint64_t* u;
  size_t u_bs;
  const uint64_t* add[2];
  uint64_t* out[2];
  const uint64_t* pinv;  // [level] P^{-1} mod q_i, [level] Shoup companions, then (as
                         // double bits) [level] P^{-1} and [level] P^{-1} / q_i
  uint32_t g;
  int32_t level;
  // batched form (out_base or tab set): batch z = 2 pair + poly writes
  // out_base + z out_bs; add_z = add_base + items[pair] add_item for poly 0
  // (gathered through phi_g), none for poly 1 or when add_base is null
  const int32_t* items;
  const uint64_t* add_base;
  size_t add_item;
  uint64_t* out_base;
  size_t out_bs;
  // inverse pass 1 only: per-modulus finishing constants [4] (conv_fin_fill)
  // replacing N^{-1}, so that the transform writes a conversion's inputs
  const uint64_t* fin;
  // batched hoisted set (tab != nullptr, batched form): output of batch z at
  // tab->out[z], pair z/2 gathered through tab->g[z/2]; add_base (items
  // null) is the one input's c0
  const SetTab* tab;
};
// the last forward NTT with the ModDown epilogue, over nbatch arrays of y
// (passes = 2: y already holds forward pass 1, as the conversion writes it)
int ntt_launch_moddown(Ctx* c, const uint64_t* y, size_t y_bs, const LimbMap& map, const NttEpi& epi, hipStream_t s,
                       int nbatch = 2, int passes = 3);
// Inverse transform whose output feeds a basis conversion: like
// ntt_launch_strided (inverse), with the last pass multiplying by the
// level's finishing constants (Ctx::d_fin) instead of N^{-1}.  passes: 3 =
// both (src -> data), 1 = pass 1 only (in place on data).
int ntt_launch_conv_in(Ctx* c, const uint64_t* src, size_t src_bs, uint64_t* data, size_t batch_stride, int nbatch,
                       const LimbMap& map, const uint64_t* fin, int passes, hipStream_t s);
// Rescale of npolys polynomials at level l (polynomial z at in + z in_bs,
// result at out + z out_bs, l - 1 limbs; out may equal in with equal
// strides) as a ModDown by the single prime q_{l-1}: inverse transform of the
// top limbs into T ([npolys][N] scratch), the conversion to q_0..q_{l-2}
// fused with the forward column pass into Y ([npolys][l-1][N] scratch), the
// forward row pass with the epilogue (c_i - y_i) q_{l-1}^{-1}.  Floor
// rounding, canonical outputs: the same residues as the textbook rescale.
int rescale_launch(Ctx* c, const uint64_t* in, size_t in_bs, uint64_t* out, size_t out_bs, int npolys, int l,
                   uint64_t* T, uint64_t* Y, hipStream_t s);
// Basis conversion fused into the forward column pass of its outputs: for
// batch z (descriptor set.d[z % zdiv], inputs in + (z / zdiv) in_bs, outputs
// out + z out_bs) every output limb out_pos[p] receives forward pass 1 of
// y_p = sum_i t_i [Qin/q_i]_p, the t_i read from in at in_pos[i].
// `target`: about how many workgroups to form when the batch is small
// (outputs are grouped accordingly; Ctx::conv_target, tuned at creation).
int conv_fwd1_launch(Ctx* c, const ConvSet& set, const uint64_t* in, size_t in_bs, uint64_t* out, size_t out_bs,
                     int nz, int zdiv, int target, const char* name, hipStream_t s);
// time the conversion kernel at the top level with a few workgroup targets
// and keep the fastest for ModUp and for ModDown
int conv_autotune(Ctx* c);
// Key inner product fused into the last forward pass of ModUp (one key
// switch): for every ext position pos < E = level + K and both key polys j,
//   u_j[pos][k] = sum_d e_d[pos][src(k)] key_d[j][mod(pos)][k] 2^-64 mod q
// with e_d the NTT form of digit d's extension (the own limb read from c1),
// src the automorphism phi_g (g = 1: identity) and the key in Montgomery form.
struct NttIp {
  const uint64_t* ext;  // [dnum][E][N] converted limbs after forward pass 1
  size_t ext_ds;
  const uint64_t* c1;   // [level][N], NTT form
  const uint64_t* key;  // [dnum][2][L+K][N], Montgomery form
  size_t key_ds, key_ps;
  uint64_t* u;          // [2][E][N]
  size_t u_ps;
  int32_t alpha, dnum, level;
  uint32_t g;
  // nonzero (needs dnum >= 2): the special-prime limbs (pos >= level) of u_0
  // and u_1 are stored after ModDown's inverse pass 2 (the pass-2
  // intermediate) instead of in NTT form
  int32_t p_inv2;
  // nonzero: ext already holds the converted limbs in NTT form (a hoisted
  // ModUp); the kernel only gathers them and no forward pass runs
  int32_t ext_ntt;
  // nonzero: ext holds the converted limbs after forward pass 1 (written by
  // the conversion kernel), so only pass 2 runs here
  int32_t ext_p1;
};
int ntt_launch_modup_ip(Ctx* c, uint64_t* ext, const LimbMap& conv, const LimbMap& outs, const NttIp& ip,
                        hipStream_t s);
constexpr int NTT_IP_MAXD = 4;  // digits the fused kernel handles (one thread group each)
// whether the fused kernel fits this ring and digit count (threads, LDS)
bool ntt_ip_supported(const Ctx* c, int dnum);
void ntt_variant_shape(int v, int* tile, int* per_thread);
// one pass of a transform: pass 2 (inverse: src -> data) or pass 1 (inverse:
// in place on data)
int ntt_launch_pass(Ctx* c, const uint64_t* src, size_t src_bs, uint64_t* data, size_t batch_stride, int nbatch,
                    const LimbMap& map, bool inverse, int pass, hipStream_t s);
// positions 0..l-1 -> q_0..q_{l-1}, positions l..l+K-1 -> p_0..p_{K-1}
LimbMap ext_map(const Ctx* c, int level);

// Workspace regions for one in-flight key switch / tensor / rescale.
struct WS {
  uint64_t *coeff, *ext, *u, *y, *t3, *rs;
};
inline WS ws_layout(const Ctx* c, uint64_t* base) {
  const size_t N = c->n, L = c->L, K = c->K, D = c->dnum(c->L);
  WS w;
  w.coeff = base;
  w.ext = w.coeff + L * N;
  w.u = w.ext + D * (L + K) * N;
  w.y = w.u + 2 * (L + K) * N;
  w.t3 = w.y + 2 * L * N;
  w.rs = w.t3 + 3 * L * N;
  return w;
}
inline size_t ws_words(const Ctx* c) {
  const size_t N = c->n, L = c->L, K = c->K, D = c->dnum(c->L);
  return N * (L + D * (L + K) + 2 * (L + K) + 2 * L + 3 * L + 2 * L);
}

// key-switching building blocks (keyswitch.hip)
int ks_modup(Ctx* c, const WS& w, const uint64_t* c1, int level, hipStream_t s);
// inner product with `key` (Montgomery form), automorphism g on the extended
// digits, ModDown, and out0 = add0[phi_g] + u0', out1 = add1 + u1'.
int ks_apply(Ctx* c, const WS& w, const uint64_t* c1, int level, const uint64_t* key, uint32_t g,
             const uint64_t* add0, const uint64_t* add1, uint64_t* out0, uint64_t* out1, hipStream_t s);
// the same key switch without a separate ModUp: ModUp's last NTT pass
// computes the inner product (NttIp), so the extended digits stay on chip
int ks_single(Ctx* c, const WS& w, const uint64_t* c1, int level, const uint64_t* key, uint32_t g,
              const uint64_t* add0, const uint64_t* add1, uint64_t* out0, uint64_t* out1, hipStream_t s);
// key cache (keys.hip): known = resident or loadable; acquire makes the key
// usable by work enqueued next on s (loading and evicting as needed, nullptr
// with the error set when that fails); note_use records its last use on s
bool key_known(const Ctx* c, int32_t id);
const uint64_t* key_acquire(Ctx* c, int32_t id, hipStream_t s);
void key_note_use(Ctx* c, int32_t id, hipStream_t s);
int key_lock(Ctx* c, int32_t id, int delta);
bool key_resident_only(const Ctx* c, int32_t id);  // uploaded, never evicted
void keys_free_all(Ctx* c);
// lane of a stream (created on first use; throws nothing, returns null on allocation failure)
Lane* lane_for(Ctx* c, hipStream_t s);
// the first n helper streams of caller stream s (created on first use);
// HE_OK or HE_EHIP
int aux_streams_for(Ctx* c, hipStream_t s, int n, hipStream_t* out);
// helpers hs[0..n) wait for the work enqueued on s so far (fork), or s waits
// for the work enqueued on each helper so far (join); HE_OK or HE_EHIP
// The constant c encoded at `scale` as an integer: llround(c * scale) (ties
// away from zero), HE_EINVAL when it does not fit 64 bits.
int const_value(double v, double scale, int64_t* out);
// out = sum_t cts[t] * vals[t] (signed integer constants, reduced per limb),
// n <= CONST_LIST_MAX terms at one level, both polynomials, in one launch;
// out's level is set, its scale is left to the caller.
constexpr int CONST_LIST_MAX = 16;
int mac_const_launch(Ctx* c, const he_ct* cts, const int64_t* vals, int n, he_ct* out, hipStream_t s);
// whether work enqueued on s is being captured into a graph
bool stream_capturing(hipStream_t s);
int stream_fork(hipStream_t s, const hipStream_t* hs, int n);
int stream_join(hipStream_t s, const hipStream_t* hs, int n);
uint64_t* lane_ct_get(Ctx* c, Lane* ln);  // null on allocation failure
int check_ct(const Ctx* c, const he_ct* x, const char* what);
int check_out(const Ctx* c, const he_ct* x, int need_level);

__global__ void k_to_mont(uint64_t* key, int M, int logn, const ModInfo* __restrict__ mods);

int32_t norm_key_id(const Ctx* c, int32_t id);
uint32_t galois_elt(const Ctx* c, int32_t r);
// psi_m^(N/2) mod q_m: a primitive fourth root of unity, the NTT value of
// X^(N/2) at the first half of the bit-reversed positions
uint64_t omega4(const Ctx* c, int m);

}  // namespace he

struct he_ctx {
  he::Ctx c;
};
