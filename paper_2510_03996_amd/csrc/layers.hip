// FHEON's secure CNN layers as CKKS schedules on the GPU ops.
//
// The schedules (rotation amounts, mask order, rescale placement) follow the
// paper's layer algorithms with one pinned reading each:
//   special conv (3x3, pad 1): Algorithm 1 rotation tree as three hoisted
//     groups, kernel vectors masked by Algorithms 2-3, input-channel sum by a
//     chain of rotations with the single key W^2 on a replicated input, block
//     masks place the out-channels;
//   generic conv (pad 0): one hoisted group of the k^2-1 tap offsets, channel
//     chain with key cs, out-channels placed by a Horner chain with key -cs;
//   striding: joint compaction of all channels in three Horner chains
//     (columns key S-1, rows key S*rs - Wo, channels key cs - Ho*Wo);
//   pooling / global pooling / FC / polynomial activation as documented in he.h.
// Every multiplicative level is rescaled once, after its last addition and
// before any rotation consumes it.
#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

namespace he {

struct LayerError {
  int code;
};

static void ck(int rc) {
  if (rc < 0) throw LayerError{rc};
}

// Layer evaluator: temporaries come from the stream's lane pool and go back
// to it (later reuse is stream-ordered after every kernel enqueued on them).
struct Ev {
  he_ctx* h;
  Ctx* c;
  he_stream s;
  Lane* lane;
  std::vector<uint64_t*> held;
  Ev(he_ctx* h_, he_stream s_) : h(h_), c(&h_->c), s(s_), lane(lane_for(&h_->c, (hipStream_t)s_)) {
    if (!lane) throw LayerError{HE_ENOMEM};
  }
  ~Ev() {
    for (uint64_t* p : held) lane->ct_pool.push_back(p);
  }
  he_ct fresh() {
    uint64_t* p = lane_ct_get(c, lane);
    if (!p) throw LayerError{HE_ENOMEM};
    held.push_back(p);
    return he_ct{p, 0, c->L, 0.0};
  }
  he_ct rot(const he_ct& x, int r) {
    he_ct o = fresh();
    ck(he_rotate(h, &x, r, &o, s));
    return o;
  }
  std::vector<he_ct> rot_hoisted(const he_ct& x, const std::vector<int>& rs) {
    if (rs.empty()) return {};  // a 1x1 kernel has no tap rotation
    std::vector<he_ct> o(rs.size());
    for (auto& t : o) t = fresh();
    ck(he_rotate_hoisted(h, &x, rs.data(), (int)rs.size(), o.data(), s));
    return o;
  }
  he_ct mul(const he_ct& x, const he_pt& p) {
    he_ct o = fresh();
    ck(he_mul_plain(h, &x, &p, &o, 0, s));
    return o;
  }
  void mac(he_ct& acc, const he_ct& x, const he_pt& p) { ck(he_mul_plain(h, &x, &p, &acc, 1, s)); }
  he_ct add(const he_ct& a, const he_ct& b) {
    he_ct o = fresh();
    ck(he_add(h, &a, &b, &o, s));
    return o;
  }
  void add_into(he_ct& acc, const he_ct& b) { ck(he_add(h, &acc, &b, &acc, s)); }
  he_ct rescale(const he_ct& x) {
    he_ct o = fresh();
    ck(he_rescale(h, &x, &o, s));
    return o;
  }
  he_ct mul_relin(const he_ct& a, const he_ct& b) {
    he_ct o = fresh();
    ck(he_mul_relin(h, &a, &b, &o, s));
    return o;
  }
  he_ct mul_const(const he_ct& x, double v, double scale) {
    he_ct o = fresh();
    ck(he_mul_const(h, &x, v, scale, &o, s));
    return o;
  }
  he_ct add_const(const he_ct& x, double v) {
    he_ct o = fresh();
    ck(he_add_const(h, &x, v, &o, s));
    return o;
  }
  static he_ct drop(const he_ct& x, int level) { return he_ct{x.data, level, x.cap, x.scale}; }
  // return a temporary's buffer to the pool (later uses are stream-ordered after
  // every kernel already enqueued on it)
  void release(const he_ct& x) {
    for (size_t i = 0; i < held.size(); i++)
      if (held[i] == x.data) {
        lane->ct_pool.push_back(held[i]);
        held[i] = held.back();
        held.pop_back();
        return;
      }
  }
  he_ct copy(const he_ct& x) {
    he_ct o = fresh();
    ck(he_drop_level(h, &x, x.level, &o, s));
    return o;
  }
  // consuming forms: the inputs are temporaries released after use
  he_ct rescale_take(const he_ct& x) {
    he_ct o = rescale(x);
    release(x);
    return o;
  }
  he_ct rot_take(const he_ct& x, int r) {
    he_ct o = rot(x, r);
    release(x);
    return o;
  }
  he_ct add_take(const he_ct& a, const he_ct& b) {
    ck(he_add(h, &a, &b, const_cast<he_ct*>(&a), s));
    release(b);
    return a;
  }
  void copy_out(const he_ct& x, he_ct* out) {
    ck(he_drop_level(h, &x, x.level, out, s));
  }
};

// sum_t ct_t (.) pt_t, one level, not rescaled
static he_ct mac_all(Ev& ev, const std::vector<he_ct>& cts, const he_pt* pts) {
  he_ct acc = ev.fresh();
  ck(he_mac_plain(ev.h, cts.data(), pts, (int)cts.size(), &acc, 0, ev.s));
  return acc;
}

// A layer's independent per-output-channel work spread over the caller's
// stream (at(0)) and up to layer_streams - 1 helper streams of it, each with
// its own evaluator (lane).  The helpers start after everything enqueued on
// the caller's stream so far; join() makes the caller's stream wait for
// them.  On destruction the helpers wait for the caller's stream, so their
// pooled temporaries (which the caller's stream may have read) are reused
// only after those reads; on an error path (no join) the host first waits
// for the helpers.  Results do not depend on the split: the work on each
// stream is the same sequence of exact modular operations.
struct Fork {
  Ev& main;
  std::vector<hipStream_t> hs;
  std::vector<Ev*> aux;
  bool joined = false;
  Fork(Ev& m, int want) : main(m) {
    const int n = std::max(0, std::min(want, 8) - 1);
    if (n == 0) return;
    hs.resize(n);
    ck(aux_streams_for(m.c, (hipStream_t)m.s, n, hs.data()));
    ck(stream_fork((hipStream_t)m.s, hs.data(), n));
    try {
      for (hipStream_t a : hs) aux.push_back(new Ev(m.h, (he_stream)a));
    } catch (...) {
      release_all();
      throw;
    }
  }
  int size() const { return 1 + (int)aux.size(); }
  Ev& at(int i) { return i == 0 ? main : *aux[i - 1]; }
  void join() {
    joined = true;  // stream_join waits on the host for a helper it cannot order
    ck(stream_join((hipStream_t)main.s, hs.data(), (int)hs.size()));
  }
  void release_all() {
    // Under graph capture the helpers are not re-forked: a later capture on
    // a helper starts from a fork of the caller's stream, which already
    // orders it after the caller's reads (and an unjoined fork would end the
    // capture with an error).
    if (!hs.empty() && !stream_capturing((hipStream_t)main.s)) {
      if (!joined)
        for (hipStream_t a : hs) hipStreamSynchronize(a);
      if (stream_fork((hipStream_t)main.s, hs.data(), (int)hs.size()) != HE_OK)
        hipStreamSynchronize((hipStream_t)main.s);
    }
    for (Ev* x : aux) delete x;
    aux.clear();
  }
  ~Fork() { release_all(); }
};

// ---------------------------------------------------------------- compaction
struct Step {
  int kind, n, key;  // kind 0 col, 1 row, 2 chan, 4 log-step column step t
  int t = 0;
};

// Stride-S extraction of outputs (S i, S j), jointly over all channels:
// columns (one chain, key S-1; or with HE_STRIDE_LOG ceil(log2 Wo) two-term
// chains with keys (S-1) 2^t), rows (key S rs - Wo), channels (key
// cs - Ho Wo), each only when it moves data.
static std::vector<Step> compaction_plan(const Ctx* c, const he_fmap& fm, int S, int Ho, int Wo, int multi = -1) {
  std::vector<Step> st;
  int T = 0;
  while ((1 << T) < Wo) T++;
  if (S > 1 && c->stride == HE_STRIDE_LOG && T > 0)
    for (int t = 0; t < T; t++) st.push_back({4, 2, (S - 1) << t, t});
  else if (S > 1)
    st.push_back({0, Wo, S - 1});
  int D = S * fm.row_stride - Wo;
  if (D != 0) st.push_back({1, Ho, D});
  int E = fm.chan_stride - Ho * Wo;
  // channels: when there are several (multi: a one-channel group of the
  // multi-channel pipeline keeps the step as one mask, so that every group
  // ends at the same level)
  if (E != 0 && (multi < 0 ? fm.channels > 1 : multi != 0)) st.push_back({2, fm.channels, E});
  return st;
}
static int compaction_masks(const std::vector<Step>& st) {
  int n = 0;
  for (auto& x : st) n += x.n;
  return n;
}

// Masked chain sum_{t<n} Rot_{t key}(v . m_t), one level.  Horner (default):
// acc = RS(v.m_{n-1}); acc = Rot_key(acc) + RS(v.m_t), t = n-2..0 (n - 1
// key switches).  Baby-step giant-step (HE_CHAIN_BSGS; the caller's masks
// m_t, t = a B + b, pre-rotated by b key): one hoisted group of the B - 1
// rotations b key of v, I_a = RS(sum_b Rot_{b key}(v) . m_{aB+b}), then
// acc = I_{A-1}; acc = Rot_{B key}(acc) + I_a: (B - 1) + (A - 1) key switches.
static void add_keys(std::vector<int>& keys, int k);
static void bsgs_split(int n, int& B, int& A) {
  B = 1;
  while (B * B < n) B++;
  A = (n + B - 1) / B;
}
static void chain_keys(const Ctx* c, std::vector<int>& keys, int n, int key) {
  if (n <= 1) return;
  if (c->chain != HE_CHAIN_BSGS) {
    add_keys(keys, key);
    return;
  }
  int B, A;
  bsgs_split(n, B, A);
  for (int b = 1; b < B; b++) add_keys(keys, b * key);
  if (A > 1) add_keys(keys, B * key);
}
static int chain_switches(const Ctx* c, int n) {
  if (n <= 1) return 0;
  if (c->chain != HE_CHAIN_BSGS) return n - 1;
  int B, A;
  bsgs_split(n, B, A);
  return (B - 1) + (A - 1);
}
static he_ct horner_masked(Ev& ev, const he_ct& v, const he_pt* m, int n, int key) {
  if (ev.c->chain != HE_CHAIN_BSGS) {
    he_ct acc = ev.rescale_take(ev.mul(v, m[n - 1]));
    for (int t = n - 2; t >= 0; t--) acc = ev.add_take(ev.rot_take(acc, key), ev.rescale_take(ev.mul(v, m[t])));
    return acc;
  }
  int B, A;
  bsgs_split(n, B, A);
  std::vector<int> offs;
  for (int b = 1; b < B; b++) offs.push_back(b * key);
  std::vector<he_ct> baby{v};
  if (!offs.empty())
    for (const he_ct& r : ev.rot_hoisted(v, offs)) baby.push_back(r);
  auto inner = [&](int a) {
    const int cnt = std::min(B, n - a * B);
    std::vector<he_ct> cts(baby.begin(), baby.begin() + cnt);
    return ev.rescale_take(mac_all(ev, cts, m + a * B));
  };
  he_ct acc = inner(A - 1);
  for (int a = A - 2; a >= 0; a--) acc = ev.add_take(ev.rot_take(acc, B * key), inner(a));
  for (size_t b = 1; b < baby.size(); b++) ev.release(baby[b]);
  return acc;
}

static he_ct compaction(Ev& ev, const he_ct& v, const he_fmap& fm, int S, int Ho, int Wo, const he_pt* masks,
                        he_fmap* out_map, int multi = -1) {
  he_ct cur = v;
  int pos = 0;
  for (const Step& st : compaction_plan(ev.c, fm, S, Ho, Wo, multi)) {
    he_ct nxt = horner_masked(ev, cur, masks + pos, st.n, st.key);
    if (pos > 0) ev.release(cur);
    cur = nxt;
    pos += st.n;
  }
  *out_map = he_fmap{fm.channels, Ho, Wo, Wo, Ho * Wo, 1};
  return cur;
}

static void add_keys(std::vector<int>& keys, int k) {
  for (int x : keys)
    if (x == k) return;
  keys.push_back(k);
}

// a plan lists its keys in he_layer_plan's 64 entries
static int plan_keys_out(he_layer_plan* pl, const std::vector<int>& keys) {
  if (keys.size() > 64) return set_error(HE_EUNSUPPORTED, "the layer needs more than 64 rotation keys");
  pl->n_keys = (int)keys.size();
  for (int i = 0; i < pl->n_keys; i++) pl->rot_keys[i] = keys[i];
  return HE_OK;
}

// ---------------------------------------------------------------- multi-channel striding
// The stride compaction of a convolution's F output channels: all at once
// (HE_STRIDE_JOINT), or the paper's multi-channel pipeline
// (HE_STRIDE_GROUP_IN): groups of g = the layer's input channels, each
// compacted jointly (group c0's channel c lands at c0 cs + c Ho Wo), then
// merged by a Horner chain with the single key g E, E = cs - Ho Wo
// (acc = z_last; acc = Rot_{gE}(acc) + z_k; no level).
static int stride_group_size(const Ctx* c, int F, int C_in) {
  return (c->stride_groups == HE_STRIDE_GROUP_IN && C_in > 0 && C_in < F) ? C_in : F;
}
// plan of the strided compaction of map f1 (F channels): keys, key switches,
// levels and masks added to the caller's counts
static void strided_plan(const Ctx* c, const he_fmap& f1, int S, int Ho, int Wo, int g, std::vector<int>& keys,
                         int& ks, int& lv, int& nmask) {
  const int F = f1.channels, multi = F > 1;
  int ngroups = 0, steps = 0;
  for (int c0 = 0; c0 < F; c0 += g, ngroups++) {
    he_fmap sub{std::min(g, F - c0), f1.height, f1.width, f1.row_stride, f1.chan_stride, 1};
    auto st = compaction_plan(c, sub, S, Ho, Wo, multi);
    for (auto& x : st) { chain_keys(c, keys, x.n, x.key); ks += chain_switches(c, x.n); }
    nmask += compaction_masks(st);
    steps = (int)st.size();
  }
  lv += steps;
  if (ngroups > 1) {
    add_keys(keys, g * (f1.chan_stride - Ho * Wo));
    ks += ngroups - 1;
  }
}
static he_ct strided(Ev& ev, const he_ct& v, const he_fmap& f1, int S, int Ho, int Wo, int g, const he_pt* masks,
                     he_fmap* out_map) {
  const int F = f1.channels, multi = F > 1;
  if (g >= F) return compaction(ev, v, f1, S, Ho, Wo, masks, out_map, multi);
  std::vector<he_ct> zs;
  int pos = 0;
  for (int c0 = 0; c0 < F; c0 += g) {
    he_fmap sub{std::min(g, F - c0), f1.height, f1.width, f1.row_stride, f1.chan_stride, 1};
    he_fmap om;
    zs.push_back(compaction(ev, v, sub, S, Ho, Wo, masks + pos, &om, multi));
    pos += compaction_masks(compaction_plan(ev.c, sub, S, Ho, Wo, multi));
  }
  he_ct acc = zs.back();
  for (int k = (int)zs.size() - 2; k >= 0; k--) {
    acc = ev.rot_take(acc, g * (f1.chan_stride - Ho * Wo));
    ev.add_into(acc, zs[k]);
    ev.release(zs[k]);
  }
  *out_map = he_fmap{F, Ho, Wo, Wo, Ho * Wo, 1};
  return acc;
}

// ---------------------------------------------------------------- conv plan
// The special schedule (Algorithm 1's rotation tree) covers 3x3 / padding 1
// on a dense square map that is replicated, or one channel in and out; any
// other padding up to (k-1)/2 uses the generic schedule, whose kernel vectors
// are zero wherever a tap's neighbour falls in the padding.
static bool conv_special(const he_fmap& fm, int F, int k, int P) {
  const int W = fm.width;
  return k == 3 && P == 1 && fm.height == W && fm.row_stride == W && fm.chan_stride == W * W &&
         (fm.reps == 2 || (fm.channels == 1 && F == 1));
}
// rotation of every tap (i, j), row-major: (i - P) rs + (j - P)
static std::vector<int> conv_taps(const he_fmap& fm, int k, int P) {
  std::vector<int> r;
  for (int i = 0; i < k; i++)
    for (int j = 0; j < k; j++) r.push_back((i - P) * fm.row_stride + (j - P));
  return r;
}

// Input-channel sum S = sum_{j < C} Rot_{j step}(A): the chain with the
// single key `step`, or (HE_CHSUM_LOG, C a power of two) doubling with keys
// 2^t step.  chsum_keys / chsum_switches describe it for the plans.
static bool chsum_log(const Ctx* c, int C) { return c->chsum == HE_CHSUM_LOG && C > 1 && (C & (C - 1)) == 0; }
static void chsum_keys(const Ctx* c, std::vector<int>& keys, int C, int step) {
  if (chsum_log(c, C))
    for (int t = 1; t < C; t *= 2) add_keys(keys, t * step);
  else if (C > 1)
    add_keys(keys, step);
}
static int chsum_switches(const Ctx* c, int C) {
  if (chsum_log(c, C)) {
    int n = 0;
    for (int t = 1; t < C; t *= 2) n++;
    return n;
  }
  return C - 1;
}
static he_ct channel_sum(Ev& ev, const he_ct& A, int C, int step) {
  he_ct S = ev.copy(A);
  if (chsum_log(ev.c, C)) {
    for (int t = 1; t < C; t *= 2) {
      he_ct R = ev.rot(S, t * step);
      ck(he_add(ev.h, &S, &R, &S, ev.s));
      ev.release(R);
    }
    return S;
  }
  he_ct T = A;
  bool own = false;  // T is A (the caller's) until the first rotation
  for (int cc = 1; cc < C; cc++) {
    he_ct T2 = ev.rot(T, step);
    if (own) ev.release(T);
    ck(he_add(ev.h, &S, &T2, &S, ev.s));
    T = T2;
    own = true;
  }
  if (own) ev.release(T);
  return S;
}

// ---------------------------------------------------------------- padding by re-layout
// Padding beyond (k-1)/2 (section "Secure Advanced Convolution With
// Padding"): the output is wider than the input, so the input is re-laid out
// as the padded tensor X_p, (C, H + 2P, W + 2P) flattened densely (row
// stride W_p = W + 2P, channel block H_p W_p), and the generic schedule runs
// on it with P = 0.  Rows are spread by one rotation amount (rs - W_p) and
// channels by another (cs - H_p W_p), each a masked chain of one level, and
// one rotation by -(P W_p + P) opens the top padding: three keys.
static he_fmap padded_map(const he_fmap& fm, int P) {
  const int Hp = fm.height + 2 * P, Wp = fm.width + 2 * P;
  return he_fmap{fm.channels, Hp, Wp, Wp, Hp * Wp, 1};
}
static bool conv_padded(const he_fmap& fm, int F, int k, int P) {
  return !conv_special(fm, F, k, P) && P > (k - 1) / 2;
}
// Step kinds here: 1 rows (n = H), 2 channels (n = C), 3 a clearing mask
// (n = 1).  Channels go first when their blocks grow enough to hold the
// rows at the input's row stride, rows first otherwise.
static int pad_plan(const he_fmap& fm, int P, std::vector<Step>& st, int* shift) {
  const he_fmap fp = padded_map(fm, P);
  const bool rows = fm.row_stride != fp.row_stride;
  const bool chan = fm.channels > 1 && fm.chan_stride != fp.chan_stride;
  const Step r{1, fm.height, fm.row_stride - fp.row_stride};
  const Step ch{2, fm.channels, fm.chan_stride - fp.chan_stride};
  st.clear();
  if (rows && chan) {
    if ((long)(fm.height - 1) * fm.row_stride + fm.width <= fp.chan_stride) st = {ch, r};
    else if ((long)(fm.height - 1) * fp.row_stride + fm.width <= fm.chan_stride) st = {r, ch};
    else return set_error(HE_EUNSUPPORTED, "the input layout leaves no room to re-lay out its rows");
  } else if (rows) {
    st = {r};
  } else if (chan) {
    st = {ch};
  } else {
    st = {Step{3, 1, 0}};
  }
  *shift = -(P * fp.row_stride + P);
  return HE_OK;
}
static int pad_mask_count(const he_fmap& fm, int F, int k, int P) {
  if (!conv_padded(fm, F, k, P)) return 0;
  std::vector<Step> st;
  int shift;
  if (pad_plan(fm, P, st, &shift)) return 0;
  return compaction_masks(st);
}
static he_ct pad_run(Ev& ev, const he_ct& x, const he_fmap& fm, int P, const he_pt* masks) {
  std::vector<Step> st;
  int shift;
  ck(pad_plan(fm, P, st, &shift));
  he_ct cur = x;
  int pos = 0;
  for (const Step& s : st) {
    he_ct nxt = horner_masked(ev, cur, masks + pos, s.n, s.key);
    if (pos > 0) ev.release(cur);
    cur = nxt;
    pos += s.n;
  }
  return ev.rot_take(cur, shift);
}

static int conv_plan_keys(const Ctx* c, const he_fmap* fm, int F, int k, int S, int P, he_layer_plan* pl,
                          std::vector<int>& keys);

static int conv_plan(const Ctx* c, const he_fmap* fm, int F, int k, int S, int P, he_layer_plan* pl) {
  std::vector<int> keys;
  const int rc = conv_plan_keys(c, fm, F, k, S, P, pl, keys);
  if (rc) return rc;
  return plan_keys_out(pl, keys);
}

// the plan without its key list, the keys appended to `keys`
static int conv_plan_keys(const Ctx* c, const he_fmap* fm, int F, int k, int S, int P, he_layer_plan* pl,
                          std::vector<int>& keys) {
  if (!fm || !pl || F < 1 || k < 1 || S < 1 || P < 0) return set_error(HE_EINVAL, "bad convolution arguments");
  const int slots = c->n / 2;
  const int C = fm->channels;
  *pl = he_layer_plan{};
  int ks = 0, lv = 0, nmask = 0;
  if (conv_special(*fm, F, k, P)) {
    const int W = fm->width;
    if (fm->reps == 2 && 2 * C * W * W != slots) return set_error(HE_EINVAL, "replicated map must fill N/2 slots");
    if (F * W * W > slots) return set_error(HE_EINVAL, "output channels do not fit the slots");
    if (S > 2) return set_error(HE_EUNSUPPORTED, "special convolution supports stride 1 or 2");
    for (int r : {-W, W, -1, 1}) add_keys(keys, r);
    ks = 8;
    lv = 1;
    if (C > 1) { chsum_keys(c, keys, C, W * W); ks += F * chsum_switches(c, C); }
    if (C > 1 || F > 1) { nmask = F; lv++; }
    he_fmap o1{F, W, W, W, W * W, (fm->reps == 2 && 2 * F * W * W == slots) ? 2 : 1};
    pl->out = o1;
    if (S > 1) {
      int Ho = (W - 1) / S + 1;
      he_fmap f1{F, W, W, W, W * W, 1};
      strided_plan(c, f1, S, Ho, Ho, stride_group_size(c, F, C), keys, ks, lv, nmask);
      pl->out = he_fmap{F, Ho, Ho, Ho, Ho * Ho, 1};
    }
    pl->n_kernel_pts = 9 * F;
  } else if (P >= 0 && P <= (k - 1) / 2) {
    const int H1 = fm->height + 2 * P - k + 1, W1 = fm->width + 2 * P - k + 1;
    if (H1 < 1 || W1 < 1) return set_error(HE_EINVAL, "kernel larger than the input");
    if (F * fm->chan_stride > slots) return set_error(HE_EINVAL, "output channels do not fit the slots");
    for (int r : conv_taps(*fm, k, P))
      if (r) add_keys(keys, r);
    ks = k * k - 1;
    lv = 1;
    if (C > 1) { chsum_keys(c, keys, C, fm->chan_stride); ks += F * chsum_switches(c, C); nmask = 1; lv++; }
    if (F > 1) { add_keys(keys, -fm->chan_stride); ks += F - 1; }
    pl->out = he_fmap{F, H1, W1, fm->row_stride, fm->chan_stride, 1};
    if (S > 1) {
      int Ho = (H1 - 1) / S + 1, Wo = (W1 - 1) / S + 1;
      he_fmap f1{F, H1, W1, fm->row_stride, fm->chan_stride, 1};
      strided_plan(c, f1, S, Ho, Wo, stride_group_size(c, F, C), keys, ks, lv, nmask);
      pl->out = he_fmap{F, Ho, Wo, Wo, Ho * Wo, 1};
    }
    pl->n_kernel_pts = k * k * F;
  } else {
    // P > (k-1)/2: X_p by re-layout, then the generic schedule with P = 0
    const he_fmap fp = padded_map(*fm, P);
    if ((long)C * fp.chan_stride > slots) return set_error(HE_EINVAL, "the padded channels do not fit the slots");
    std::vector<Step> st;
    int shift, rc;
    if ((rc = pad_plan(*fm, P, st, &shift))) return rc;
    for (auto& x : st) { chain_keys(c, keys, x.n, x.key); ks += chain_switches(c, x.n); lv++; }
    nmask = compaction_masks(st);
    add_keys(keys, shift);
    ks++;
    he_layer_plan sub;
    if ((rc = conv_plan_keys(c, &fp, F, k, S, 0, &sub, keys))) return rc;
    ks += sub.key_switches;
    lv += sub.levels;
    nmask += sub.n_mask_pts;
    pl->out = sub.out;
    pl->n_kernel_pts = sub.n_kernel_pts;
  }
  pl->n_mask_pts = nmask;
  pl->levels = lv;
  pl->key_switches = ks;
  return HE_OK;
}

static he_ct conv_run(Ev& ev, const he_ct& x, const he_fmap& fm, int F, int k, int S, int P, const he_pt* kern,
                      const he_pt* masks, he_fmap* out_map) {
  const int C = fm.channels;
  if (conv_padded(fm, F, k, P)) {
    const int npad = pad_mask_count(fm, F, k, P);
    he_ct xp = pad_run(ev, x, fm, P, masks);
    he_ct y = conv_run(ev, xp, padded_map(fm, P), F, k, S, 0, kern, masks + npad, out_map);
    ev.release(xp);
    return y;
  }
  if (conv_special(fm, F, k, P)) {
    const int W = fm.width;
    auto g1 = ev.rot_hoisted(x, {-W, W, -1, 1});  // r1, r7, r3, r5
    auto g2 = ev.rot_hoisted(g1[0], {-1, 1});     // r0, r2
    auto g3 = ev.rot_hoisted(g1[1], {-1, 1});     // r6, r8
    std::vector<he_ct> taps = {g2[0], g1[0], g2[1], g1[2], x, g1[3], g3[0], g1[1], g3[1]};
    const bool place = C > 1 || F > 1;
    he_ct y{};
    {
      // output channel f on stream f mod K; per-stream partial sums of the
      // placed channels, added on the caller's stream
      Fork fk(ev, place ? std::min(ev.c->streams_for_ring(), F) : 1);
      const int K = fk.size();
      std::vector<he_ct> part(K);
      std::vector<bool> has(K, false);
      for (int f = 0; f < F; f++) {
        Ev& e = fk.at(f % K);
        he_ct A = e.rescale_take(mac_all(e, taps, kern + 9 * f));
        he_ct Ssum = A;
        if (C > 1) {
          // S_f = A_f + Rot_{W^2}(A_f) + Rot_{2 W^2}(A_f) + ...
          Ssum = channel_sum(e, A, C, W * W);
          e.release(A);
        }
        if (place) {
          if (!has[f % K]) part[f % K] = e.mul(Ssum, masks[f]);
          else e.mac(part[f % K], Ssum, masks[f]);
          has[f % K] = true;
          e.release(Ssum);
        } else {
          y = Ssum;
        }
      }
      fk.join();
      if (place) {
        y = part[0];
        for (int k = 1; k < K; k++)
          if (has[k]) ev.add_into(y, part[k]);
      }
    }
    int mpos = 0;
    if (place) {
      y = ev.rescale_take(y);
      mpos = F;
    }
    for (int t = 0; t < 9; t++)
      if (t != 4) ev.release(taps[t]);
    const int slots = ev.c->n / 2;
    *out_map = he_fmap{F, W, W, W, W * W, (fm.reps == 2 && 2 * F * W * W == slots) ? 2 : 1};
    if (S == 1) return y;
    int Ho = (W - 1) / S + 1;
    he_ct z = strided(ev, y, he_fmap{F, W, W, W, W * W, 1}, S, Ho, Ho, stride_group_size(ev.c, F, C), masks + mpos,
                      out_map);
    ev.release(y);
    return z;
  }
  // generic: taps (i, j) row-major, rotated by (i - P) rs + (j - P) (one hoisted group)
  const std::vector<int> tap_rot = conv_taps(fm, k, P);
  std::vector<int> offs;
  for (int r : tap_rot)
    if (r) offs.push_back(r);
  auto rots = ev.rot_hoisted(x, offs);
  std::vector<he_ct> taps;
  size_t next = 0;
  for (int r : tap_rot) taps.push_back(r ? rots[next++] : x);
  const int cs = fm.chan_stride;
  he_ct acc{};
  {
    // per-channel terms (output channel f on stream f mod K), then the
    // placement chain on the caller's stream
    Fork fk(ev, std::min(ev.c->streams_for_ring(), F));
    const int K = fk.size();
    std::vector<he_ct> terms(F);
    for (int f = F - 1; f >= 0; f--) {
      Ev& e = fk.at(f % K);
      he_ct A = e.rescale_take(mac_all(e, taps, kern + k * k * f));
      he_ct term = A;
      if (C > 1) {
        he_ct sum = channel_sum(e, A, C, cs);
        e.release(A);
        term = e.rescale_take(e.mul(sum, masks[0]));
        e.release(sum);
      }
      if (K == 1) {  // fold at once (one term alive at a time)
        acc = (f == F - 1) ? term : ev.add_take(ev.rot_take(acc, -cs), term);
      } else {
        terms[f] = term;
      }
    }
    fk.join();
    if (K > 1) {
      // rot_take returns only the caller evaluator's own temporaries
      acc = terms[F - 1];
      for (int f = F - 2; f >= 0; f--) {
        acc = ev.rot_take(acc, -cs);
        ev.add_into(acc, terms[f]);
      }
    }
  }
  for (auto& r : rots) ev.release(r);
  const int H1 = fm.height + 2 * P - k + 1, W1 = fm.width + 2 * P - k + 1;
  *out_map = he_fmap{F, H1, W1, fm.row_stride, cs, 1};
  if (S == 1) return acc;
  int Ho = (H1 - 1) / S + 1, Wo = (W1 - 1) / S + 1;
  he_ct z = strided(ev, acc, he_fmap{F, H1, W1, fm.row_stride, cs, 1}, S, Ho, Wo, stride_group_size(ev.c, F, C),
                    masks + (C > 1 ? 1 : 0),
                       out_map);
  ev.release(acc);
  return z;
}

// ---------------------------------------------------------------- pooling plan
// The pooling special case (section "Secure Average Pooling Layer"): a
// window covering the whole (square, dense) channel gives one value per
// channel, i.e. the global schedule: the channel's sum by log-step rotations,
// 1/k^2 and each channel's first value gathered with one key.
static bool pool_whole_channel(const he_fmap& fm, int k) {
  return k > 0 && k == fm.height && k == fm.width && fm.row_stride == fm.width &&
         fm.chan_stride == fm.height * fm.width && (fm.chan_stride & (fm.chan_stride - 1)) == 0;
}

static int pool_plan(const Ctx* c, const he_fmap* fm, int k, int S, he_layer_plan* pl) {
  if (!fm || !pl || k < 0 || S < 1) return set_error(HE_EINVAL, "bad pooling arguments");
  if (pool_whole_channel(*fm, k)) k = 0;
  *pl = he_layer_plan{};
  std::vector<int> keys;
  int ks = 0;
  if (k == 0) {
    const int cs = fm->chan_stride;
    if (fm->row_stride != fm->width || cs != fm->height * fm->width || (cs & (cs - 1)))
      return set_error(HE_EUNSUPPORTED, "global pooling needs dense power-of-two channel blocks");
    for (int t = 1; t < cs; t <<= 1) { add_keys(keys, t); ks++; }
    chain_keys(c, keys, fm->channels, cs - 1);
    ks += chain_switches(c, fm->channels);
    pl->n_mask_pts = fm->channels;
    pl->levels = 1;
    pl->out = he_fmap{fm->channels, 1, 1, 1, 1, 1};
  } else {
    const int H1 = fm->height - k + 1, W1 = fm->width - k + 1;
    if (H1 < 1 || W1 < 1) return set_error(HE_EINVAL, "window larger than the input");
    for (int i = 0; i < k; i++)
      for (int j = 0; j < k; j++)
        if (i || j) { add_keys(keys, i * fm->row_stride + j); ks++; }
    if (S == 1) {
      pl->n_mask_pts = 1;
      pl->levels = 1;
      pl->out = he_fmap{fm->channels, H1, W1, fm->row_stride, fm->chan_stride, 1};
    } else {
      int Ho = (fm->height - k) / S + 1, Wo = (fm->width - k) / S + 1;
      he_fmap f1{fm->channels, H1, W1, fm->row_stride, fm->chan_stride, 1};
      auto st = compaction_plan(c, f1, S, Ho, Wo);
      for (auto& x : st) { chain_keys(c, keys, x.n, x.key); ks += chain_switches(c, x.n); }
      pl->n_mask_pts = compaction_masks(st);
      pl->levels = (int)st.size();
      pl->out = he_fmap{fm->channels, Ho, Wo, Wo, Ho * Wo, 1};
    }
  }
  pl->key_switches = ks;
  return plan_keys_out(pl, keys);
}

static he_ct pool_run(Ev& ev, const he_ct& x, const he_fmap& fm, int k, int S, const he_pt* masks,
                      he_fmap* out_map) {
  if (k == 0 || pool_whole_channel(fm, k)) {
    const int cs = fm.chan_stride;
    he_ct Ssum = ev.copy(x);
    for (int t = 1; t < cs; t <<= 1) Ssum = ev.add_take(Ssum, ev.rot(Ssum, t));
    *out_map = he_fmap{fm.channels, 1, 1, 1, 1, 1};
    he_ct y = horner_masked(ev, Ssum, masks, fm.channels, cs - 1);
    ev.release(Ssum);
    return y;
  }
  std::vector<int> offs;
  for (int i = 0; i < k; i++)
    for (int j = 0; j < k; j++)
      if (i || j) offs.push_back(i * fm.row_stride + j);
  auto rots = ev.rot_hoisted(x, offs);
  he_ct s = ev.add(x, rots[0]);
  for (size_t t = 1; t < rots.size(); t++) ev.add_into(s, rots[t]);
  for (auto& r : rots) ev.release(r);
  const int H1 = fm.height - k + 1, W1 = fm.width - k + 1;
  he_fmap f1{fm.channels, H1, W1, fm.row_stride, fm.chan_stride, 1};
  if (S == 1) {
    *out_map = f1;
    return ev.rescale_take(ev.mul(s, masks[0]));
  }
  int Ho = (fm.height - k) / S + 1, Wo = (fm.width - k) / S + 1;
  he_ct z = compaction(ev, s, f1, S, Ho, Wo, masks, out_map);
  ev.release(s);
  return z;
}

static int fc_plan_impl(const Ctx* c, int n_in, int n_out, he_layer_plan* pl) {
  if (!pl || n_in < 1 || (n_in & (n_in - 1)) || n_out < 1)
    return set_error(HE_EINVAL, "n_in must be a power of two and n_out >= 1");
  *pl = he_layer_plan{};
  std::vector<int> keys;
  int ks = 0;
  if (c->fc == HE_FC_DIAG) {
    if (n_out > n_in) return set_error(HE_EINVAL, "the diagonal form needs n_out <= n_in");
    int B, A;
    bsgs_split(n_in, B, A);
    add_keys(keys, -n_in);
    for (int b = 1; b < B; b++) add_keys(keys, b);
    if (A > 1) add_keys(keys, B);
    ks = 1 + (B - 1) + (A - 1);
    pl->n_kernel_pts = n_in;
    pl->n_mask_pts = 0;
    pl->levels = 1;
    pl->key_switches = ks;
    pl->out = he_fmap{n_out, 1, 1, 1, 1, 1};
    return plan_keys_out(pl, keys);
  }
  for (int t = 1; t < n_in; t <<= 1) { add_keys(keys, t); ks += n_out; }
  if (n_out > 1) { add_keys(keys, -1); ks += n_out - 1; }
  pl->n_kernel_pts = n_out;
  pl->n_mask_pts = 1;
  pl->levels = 2;
  pl->key_switches = ks;
  pl->out = he_fmap{n_out, 1, 1, 1, 1, 1};
  return plan_keys_out(pl, keys);
}

// ---------------------------------------------------------------- Chebyshev secure ReLU
// Baby-step giant-step evaluation of f = sum_j a_j T_j (a_0 = c_0 / 2): the
// series is divided recursively by giant steps T_K (K = 8 2^m, the largest
// not above the degree; T_{K+i} = 2 T_K T_i - T_{K-i}) down to leaves of
// degree below 8, and every subtree is evaluated directly onto a target
// level and scale.
constexpr int CHEB_BABY = 8;

struct ChebNode {
  int K = 0;              // 0: leaf
  std::vector<double> a;  // leaf coefficients
  int q = -1, r = -1;     // children (quotient, remainder)
};

static int cheb_build(std::vector<ChebNode>& t, std::vector<double> a) {
  int d = (int)a.size() - 1;
  while (d > 0 && a[d] == 0.0) d--;
  a.resize(d + 1);
  const int id = (int)t.size();
  t.emplace_back();
  if (d < CHEB_BABY) {
    t[id].a = a;
    return id;
  }
  int K = CHEB_BABY;
  while (2 * K <= d) K *= 2;
  std::vector<double> q(d - K + 1), r(a.begin(), a.begin() + K);
  q[0] = a[K];
  for (int i = 1; i <= d - K; i++) q[i] = 2.0 * a[K + i];
  for (int i = 2 * K - d; i < K; i++) r[i] = a[i] - a[2 * K - i];
  const int qi = cheb_build(t, q);
  const int ri = cheb_build(t, r);
  t[id].K = K;
  t[id].q = qi;
  t[id].r = ri;
  return id;
}

static std::vector<ChebNode> cheb_tree(const double* cf, int degree) {
  std::vector<double> a(cf, cf + degree + 1);
  a[0] = a[0] / 2.0;
  std::vector<ChebNode> t;
  cheb_build(t, a);
  return t;
}

static int cheb_depth(int j) { return j <= 1 ? 0 : 32 - __builtin_clz((unsigned)(j - 1)); }

// T_j (j >= 1) the evaluation computes, ascending: the leaves' nonzero terms,
// T_1, the giant steps and, recursively, the factors of the product rule
// T_{2k} = 2 T_k^2 - 1, T_{2k+1} = 2 T_k T_{k+1} - T_1.
static std::vector<int> cheb_terms(const std::vector<ChebNode>& tree) {
  int maxj = 1;
  for (auto& n : tree) maxj = std::max(maxj, n.K ? n.K : (int)n.a.size() - 1);
  std::vector<char> need(maxj + 1, 0);
  std::vector<int> stack{1};
  for (auto& n : tree) {
    if (n.K) stack.push_back(n.K);
    else
      for (int j = 1; j < (int)n.a.size(); j++)
        if (n.a[j] != 0.0) stack.push_back(j);
  }
  while (!stack.empty()) {
    const int j = stack.back();
    stack.pop_back();
    if (need[j]) continue;
    need[j] = 1;
    if (j >= 2) {
      stack.push_back(j / 2);
      if (j % 2) stack.push_back(j / 2 + 1);
    }
  }
  std::vector<int> out;
  for (int j = 1; j <= maxj; j++)
    if (need[j]) out.push_back(j);
  return out;
}

// highest level subtree `id` can be evaluated onto (T_j at level top - depth(j))
static int cheb_allowed(const std::vector<ChebNode>& t, int id, int top) {
  const ChebNode& n = t[id];
  if (!n.K) {
    int lv = INT32_MAX;
    for (int j = 1; j < (int)n.a.size(); j++)
      if (n.a[j] != 0.0) lv = std::min(lv, top - cheb_depth(j) - 1);
    return lv == INT32_MAX ? top - 1 : lv;
  }
  return std::min(top - cheb_depth(n.K) - 1, std::min(cheb_allowed(t, n.q, top) - 1, cheb_allowed(t, n.r, top)));
}

static int cheb_plan_impl(const double* cf, int degree, int masked, int* levels, int* relins) {
  if (!cf || degree < 1 || degree > HE_CHEB_MAX_DEGREE) return set_error(HE_EINVAL, "degree must be in [1, 255]");
  bool any = false;
  for (int j = 1; j <= degree; j++) any = any || cf[j] != 0.0;
  if (!any) return set_error(HE_EINVAL, "every coefficient of degree >= 1 is zero");
  const std::vector<ChebNode> tree = cheb_tree(cf, degree);
  int nodes = 0;
  for (auto& n : tree) nodes += n.K != 0;
  *levels = (masked ? 1 : 0) - cheb_allowed(tree, 0, 0);
  *relins = (int)cheb_terms(tree).size() - 1 + nodes;
  return HE_OK;
}

// c v at `level` with tracked scale `scale`: v dropped to level + 1, times c
// encoded at sigma = scale q / s_v (q the prime the rescale divides by),
// rescaled; the tracked scale is set to `scale` (the product's, up to the
// rounding of sigma).
static he_ct cheb_lift(Ev& ev, const he_ct& v, int level, double scale, double c) {
  const double q = (double)ev.c->mod[level];
  he_ct t = ev.rescale_take(ev.mul_const(Ev::drop(v, level + 1), c, scale * q / v.scale));
  t.scale = scale;
  return t;
}

// subtree `id` evaluated onto (level, scale): a leaf with one rescale,
// RS(sum_j a_j T_j) + a_0 (ascending j; T_1 times 0 if it has none): each
// T_j dropped to level + 1 times a_j encoded at scale q / s(T_j), every
// product recorded at scale q (q the prime the rescale removes), summed,
// rescaled and recorded at `scale`; a node as RS(Relin(q' T_K)) with scale
// `scale` plus r', q' evaluated one level higher at scale q_level / s(T_K)
// times `scale`, r' onto (level, scale)
static he_ct cheb_eval_node(Ev& ev, const std::vector<ChebNode>& t, int id, const std::vector<he_ct>& T, int level,
                            double scale) {
  const ChebNode& n = t[id];
  if (!n.K) {
    // the products and their sum in one pass (a leaf has fewer than eight
    // terms): the same residues as one constant product per term, added
    const double q = (double)ev.c->mod[level];
    std::vector<he_ct> terms;
    std::vector<int64_t> vals;
    for (int j = 1; j < (int)n.a.size(); j++) {
      if (n.a[j] == 0.0) continue;
      const he_ct v = Ev::drop(T[j], level + 1);
      int64_t x = 0;
      ck(const_value(n.a[j], scale * q / v.scale, &x));
      terms.push_back(v);
      vals.push_back(x);
    }
    if (terms.empty()) {
      const he_ct v = Ev::drop(T[1], level + 1);
      int64_t x = 0;
      ck(const_value(0.0, scale * q / v.scale, &x));
      terms.push_back(v);
      vals.push_back(x);
    }
    he_ct acc = ev.fresh();
    ck(mac_const_launch(ev.c, terms.data(), vals.data(), (int)terms.size(), &acc, (hipStream_t)ev.s));
    acc.scale = scale * q;
    he_ct r = ev.rescale_take(acc);
    r.scale = scale;
    he_ct y = ev.add_const(r, n.a[0]);
    ev.release(r);
    return y;
  }
  const double sigma = scale * (double)ev.c->mod[level] / T[n.K].scale;
  he_ct qc = cheb_eval_node(ev, t, n.q, T, level + 1, sigma);
  he_ct p = ev.rescale_take(ev.mul_relin(qc, Ev::drop(T[n.K], level + 1)));
  ev.release(qc);
  p.scale = scale;
  he_ct rc = cheb_eval_node(ev, t, n.r, T, level, scale);
  return ev.add_take(p, rc);
}

// ---------------------------------------------------------------- plaintext recipes
// The real slot vectors a layer multiplies by, built on the host in the
// order and number the layer's plan gives (the model owner's weight
// preprocessing).  V is [count][slots]; every builder appends.
using Vecs = std::vector<std::vector<double>>;

static std::vector<double> zeros(int slots) { return std::vector<double>((size_t)slots, 0.0); }

// Rot_r moves slot i + r to slot i: the vector a rotation by r would give
static std::vector<double> rotated(const std::vector<double>& m, long r) {
  const long n = (long)m.size();
  std::vector<double> o(m.size());
  for (long i = 0; i < n; i++) o[i] = m[(size_t)(((i + r) % n + n) % n)];
  return o;
}

// masks of a masked chain with key `key`: as given (Horner), or mask t = a B + b
// rotated by b key (baby-step giant-step)
static void chain_vectors(const Ctx* c, Vecs& out, Vecs v, int key) {
  if (c->chain == HE_CHAIN_BSGS && v.size() > 1) {
    int B, A;
    bsgs_split((int)v.size(), B, A);
    for (size_t t = 0; t < v.size(); t++) v[t] = rotated(v[t], (long)(t % B) * key);
  }
  for (auto& x : v) out.push_back(std::move(x));
}

// stride-S extraction masks of outputs (S i, S j) of map fm (compaction_plan)
// (channels c0 .. c0 + channels - 1 of the map: a group of the multi-channel pipeline)
static void compaction_vectors(const Ctx* c, Vecs& out, const he_fmap& fm, int S, int Ho, int Wo, double col_scale,
                               int c0 = 0, int multi = -1) {
  const int slots = c->n / 2;
  for (const Step& st : compaction_plan(c, fm, S, Ho, Wo, multi)) {
    Vecs v;
    for (int t = 0; t < st.n; t++) {
      std::vector<double> m = zeros(slots);
      for (int ch = c0; ch < c0 + fm.channels; ch++) {
        if (st.kind == 4) {
          // after steps < st.t column j sits at S (j - b) + b, b = j mod 2^st.t;
          // mask 0 holds the j with bit st.t clear, mask 1 those with it set
          const int lo = (1 << st.t) - 1;
          for (int i = 0; i < Ho; i++)
            for (int j = 0; j < Wo; j++)
              if (((j >> st.t) & 1) == t)
                m[(size_t)ch * fm.chan_stride + (size_t)S * i * fm.row_stride + S * (j & ~lo) + (j & lo)] =
                    st.t == 0 ? col_scale : 1.0;
        } else if (st.kind == 0) {
          for (int i = 0; i < Ho; i++) m[(size_t)ch * fm.chan_stride + (size_t)S * i * fm.row_stride + S * t] = col_scale;
        } else if (st.kind == 1) {
          const size_t base = (size_t)ch * fm.chan_stride + (size_t)S * t * fm.row_stride;
          for (int j = 0; j < Wo; j++) m[base + j] = 1.0;
        } else if (ch == c0 + t) {
          for (int j = 0; j < Ho * Wo; j++) m[(size_t)ch * fm.chan_stride + j] = 1.0;
        }
      }
      v.push_back(std::move(m));
    }
    chain_vectors(c, out, std::move(v), st.key);
  }
}

// the convolution's stride masks: each group of the multi-channel pipeline in turn
static void strided_vectors(const Ctx* c, Vecs& out, const he_fmap& f1, int S, int Ho, int Wo, int g) {
  const int F = f1.channels;
  for (int c0 = 0; c0 < F; c0 += g)
    compaction_vectors(c, out, he_fmap{std::min(g, F - c0), f1.height, f1.width, f1.row_stride, f1.chan_stride, 1}, S,
                       Ho, Wo, 1.0, c0, F > 1);
}

// convolution: kernel vectors [f][tap], then masks, then (bias) the bias
// vector on the output layout.  K is [F][C][k][k].
static int conv_vectors(const Ctx* c, const he_fmap& fm, int F, int k, int S, int P, const double* K, const double* bias,
                        Vecs& out) {
  he_layer_plan pl;
  int rc;
  if ((rc = conv_plan(c, &fm, F, k, S, P, &pl))) return rc;
  const int slots = c->n / 2, C = fm.channels;
  auto w = [&](int f, int ch, int i, int j) { return K[(((size_t)f * C + ch) * k + i) * k + j]; };
  if (conv_padded(fm, F, k, P)) {
    // re-layout masks on the layout each step sees, then the P = 0 vectors on X_p
    std::vector<Step> st;
    int shift;
    if ((rc = pad_plan(fm, P, st, &shift))) return rc;
    Vecs pads;
    int rs = fm.row_stride, cs = fm.chan_stride;
    const he_fmap fp = padded_map(fm, P);
    for (const Step& x : st) {
      Vecs v;
      for (int t = 0; t < x.n; t++) {
        std::vector<double> m = zeros(slots);
        for (int ch = 0; ch < C; ch++)
          for (int y = 0; y < fm.height; y++) {
            if ((x.kind == 2 && ch != t) || (x.kind == 1 && y != t)) continue;
            const size_t base = (size_t)ch * cs + (size_t)y * rs;
            for (int j = 0; j < fm.width; j++) m[base + j] = 1.0;
          }
        v.push_back(std::move(m));
      }
      chain_vectors(c, pads, std::move(v), x.key);
      if (x.kind == 2) cs = fp.chan_stride;
      if (x.kind == 1) rs = fp.row_stride;
    }
    Vecs rest;
    if ((rc = conv_vectors(c, fp, F, k, S, 0, K, bias, rest))) return rc;
    const size_t nk = (size_t)k * k * F;
    for (size_t i = 0; i < nk; i++) out.push_back(std::move(rest[i]));
    for (auto& m : pads) out.push_back(std::move(m));
    for (size_t i = nk; i < rest.size(); i++) out.push_back(std::move(rest[i]));
    return HE_OK;
  }
  if (conv_special(fm, F, k, P)) {
    const int W = fm.width, WW = W * W;
    for (int f = 0; f < F; f++)
      for (int tap = 0; tap < 9; tap++) {
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        std::vector<double> v = zeros(slots);
        for (int b = 0; b < fm.reps * C; b++)
          for (int y = 0; y < W; y++)
            for (int x = 0; x < W; x++)
              if (y + dy >= 0 && y + dy < W && x + dx >= 0 && x + dx < W)
                v[(size_t)b * WW + y * W + x] = w(f, b % C, dy + 1, dx + 1);
        out.push_back(std::move(v));
      }
    const int reps1 = (fm.reps == 2 && 2 * F * WW == slots) ? 2 : 1;
    if (F > 1 || C > 1)
      for (int f = 0; f < F; f++) {
        std::vector<double> m = zeros(slots);
        for (int r = 0; r < reps1; r++)
          for (int t = 0; t < WW; t++) m[(size_t)(r * F + f) * WW + t] = 1.0;
        out.push_back(std::move(m));
      }
    if (S > 1) {
      const int Ho = (W - 1) / S + 1;
      strided_vectors(c, out, he_fmap{F, W, W, W, WW, 1}, S, Ho, Ho, stride_group_size(c, F, C));
    }
  } else {
    const int H1 = fm.height + 2 * P - k + 1, W1 = fm.width + 2 * P - k + 1;
    for (int f = 0; f < F; f++)
      for (int i = 0; i < k; i++)
        for (int j = 0; j < k; j++) {
          std::vector<double> v = zeros(slots);
          const int x0 = std::max(0, P - j), x1 = std::min(W1, fm.width + P - j);
          for (int ch = 0; ch < C; ch++)
            for (int y = 0; y < H1; y++)
              if (y + i - P >= 0 && y + i - P < fm.height)
                for (int x = x0; x < x1; x++) v[(size_t)ch * fm.chan_stride + (size_t)y * fm.row_stride + x] = w(f, ch, i, j);
          out.push_back(std::move(v));
        }
    if (C > 1) {
      std::vector<double> m = zeros(slots);
      for (int y = 0; y < H1; y++)
        for (int x = 0; x < W1; x++) m[(size_t)y * fm.row_stride + x] = 1.0;
      out.push_back(std::move(m));
    }
    if (S > 1) {
      const int Ho = (H1 - 1) / S + 1, Wo = (W1 - 1) / S + 1;
      strided_vectors(c, out, he_fmap{F, H1, W1, fm.row_stride, fm.chan_stride, 1}, S, Ho, Wo,
                      stride_group_size(c, F, C));
    }
  }
  if (bias) {
    const he_fmap& o = pl.out;
    std::vector<double> v = zeros(slots);
    for (int r = 0; r < o.reps; r++)
      for (int f = 0; f < F; f++)
        for (int y = 0; y < o.height; y++)
          for (int x = 0; x < o.width; x++)
            v[(size_t)(r * F + f) * o.chan_stride + (size_t)y * o.row_stride + x] = bias[f];
    out.push_back(std::move(v));
  }
  return HE_OK;
}

static int pool_vectors(const Ctx* c, const he_fmap& fm, int k, int S, Vecs& out) {
  he_layer_plan pl;
  int rc;
  if ((rc = pool_plan(c, &fm, k, S, &pl))) return rc;
  const int slots = c->n / 2;
  if (k == 0 || pool_whole_channel(fm, k)) {
    Vecs v;
    for (int ch = 0; ch < fm.channels; ch++) {
      std::vector<double> m = zeros(slots);
      m[(size_t)ch * fm.chan_stride] = 1.0 / ((double)fm.height * fm.width);
      v.push_back(std::move(m));
    }
    chain_vectors(c, out, std::move(v), fm.chan_stride - 1);
    return HE_OK;
  }
  const int H1 = fm.height - k + 1, W1 = fm.width - k + 1;
  const double inv = 1.0 / ((double)k * k);
  if (S == 1) {
    std::vector<double> m = zeros(slots);
    for (int ch = 0; ch < fm.channels; ch++)
      for (int y = 0; y < H1; y++)
        for (int x = 0; x < W1; x++) m[(size_t)ch * fm.chan_stride + (size_t)y * fm.row_stride + x] = inv;
    out.push_back(std::move(m));
    return HE_OK;
  }
  const int Ho = (fm.height - k) / S + 1, Wo = (fm.width - k) / S + 1;
  compaction_vectors(c, out, he_fmap{fm.channels, H1, W1, fm.row_stride, fm.chan_stride, 1}, S, Ho, Wo, inv);
  return HE_OK;
}

// fully connected: rows W_k then e_0 (rows form), or the n_in diagonals
// W[j][(j + d) mod n_in] rotated by -(d / B) B (diagonal form); then the bias
// in slots 0..n_out-1 when given.  Wm is [n_out][n_in].
static int fc_vectors(const Ctx* c, int n_in, int n_out, const double* Wm, const double* bias, Vecs& out) {
  he_layer_plan pl;
  int rc;
  if ((rc = fc_plan_impl(c, n_in, n_out, &pl))) return rc;
  const int slots = c->n / 2;
  if (n_in > slots) return set_error(HE_EINVAL, "n_in exceeds the slots");
  if (c->fc == HE_FC_DIAG) {
    int B, A;
    bsgs_split(n_in, B, A);
    for (int d = 0; d < n_in; d++) {
      std::vector<double> v = zeros(slots);
      for (int j = 0; j < n_out; j++) v[j] = Wm[(size_t)j * n_in + (j + d) % n_in];
      out.push_back(rotated(v, -(long)(d / B) * B));
    }
  } else {
    for (int kk = 0; kk < n_out; kk++) {
      std::vector<double> v = zeros(slots);
      for (int j = 0; j < n_in; j++) v[j] = Wm[(size_t)kk * n_in + j];
      out.push_back(std::move(v));
    }
    std::vector<double> e0 = zeros(slots);
    e0[0] = 1.0;
    out.push_back(std::move(e0));
  }
  if (bias) {
    std::vector<double> v = zeros(slots);
    for (int j = 0; j < n_out; j++) v[j] = bias[j];
    out.push_back(std::move(v));
  }
  return HE_OK;
}

}  // namespace he

using namespace he;

template <class F>
static int guarded(F&& f) {
  try {
    return f();
  } catch (const LayerError& e) {
    return e.code;
  } catch (const std::bad_alloc&) {
    return set_error(HE_ENOMEM, "host allocation failed");
  }
}

static int check_pts(const Ctx* c, const he_pt* p, int n, int level, const char* what) {
  if (n > 0 && !p) return set_error(HE_EINVAL, std::string(what) + ": null plaintext array");
  for (int i = 0; i < n; i++)
    if (!p[i].data || p[i].level < level)
      return set_error(HE_ELEVEL, std::string(what) + ": plaintext with too few limbs");
  (void)c;
  return HE_OK;
}


extern "C" {

int he_ctx_stride_groups(he_ctx* h, int mode) {
  if (!h) return set_error(HE_EINVAL, "null context");
  if (mode != HE_STRIDE_JOINT && mode != HE_STRIDE_GROUP_IN) return set_error(HE_EINVAL, "unknown stride grouping");
  h->c.stride_groups = mode;
  return HE_OK;
}

int he_ctx_striding(he_ctx* h, int mode) {
  if (!h) return set_error(HE_EINVAL, "null context");
  if (mode != HE_STRIDE_EXTRACT && mode != HE_STRIDE_LOG) return set_error(HE_EINVAL, "unknown striding mode");
  h->c.stride = mode;
  return HE_OK;
}

int he_ctx_mask_chains(he_ctx* h, int mode) {
  if (!h) return set_error(HE_EINVAL, "null context");
  if (mode != HE_CHAIN_HORNER && mode != HE_CHAIN_BSGS) return set_error(HE_EINVAL, "unknown chain mode");
  h->c.chain = mode;
  return HE_OK;
}

int he_ctx_conv_channel_sum(he_ctx* h, int mode) {
  if (!h) return set_error(HE_EINVAL, "null context");
  if (mode != HE_CHSUM_CHAIN && mode != HE_CHSUM_LOG) return set_error(HE_EINVAL, "unknown channel-sum mode");
  h->c.chsum = mode;
  return HE_OK;
}

int he_conv2d_plan(const he_ctx* h, const he_fmap* in_map, int out_ch, int kernel, int stride, int padding,
                   he_layer_plan* plan) {
  if (!h) return set_error(HE_EINVAL, "null context");
  return conv_plan(&h->c, in_map, out_ch, kernel, stride, padding, plan);
}

int he_conv2d(he_ctx* h, const he_ct* in, const he_fmap* in_map, int out_ch, int kernel, int stride, int padding,
              const he_pt* kernel_pts, int n_kernel_pts, const he_pt* mask_pts, int n_mask_pts, const he_pt* bias_pt,
              he_ct* out, he_fmap* out_map, he_stream s) {
  if (!h || !out_map) return set_error(HE_EINVAL, "null argument");
  Ctx* c = &h->c;
  he_layer_plan pl;
  int rc;
  if ((rc = check_ct(c, in, "in"))) return rc;
  if ((rc = conv_plan(c, in_map, out_ch, kernel, stride, padding, &pl))) return rc;
  if (n_kernel_pts != pl.n_kernel_pts || n_mask_pts != pl.n_mask_pts)
    return set_error(HE_EINVAL, "plaintext counts differ from the layer plan");
  if (in->level <= pl.levels) return set_error(HE_ELEVEL, "not enough levels for the convolution");
  if ((rc = check_out(c, out, in->level - pl.levels))) return rc;
  if ((rc = check_pts(c, kernel_pts, n_kernel_pts, in->level, "kernel_pts"))) return rc;
  const int npad = pad_mask_count(*in_map, out_ch, kernel, padding);  // used at the input level
  if ((rc = check_pts(c, mask_pts, npad, in->level, "mask_pts")) ||
      (rc = check_pts(c, mask_pts + npad, n_mask_pts - npad, in->level - pl.levels + 1, "mask_pts")))
    return rc;
  if (bias_pt && (rc = check_pts(c, bias_pt, 1, in->level - pl.levels, "bias_pt"))) return rc;
  for (int i = 0; i < pl.n_keys; i++)
    if (!key_known(c, pl.rot_keys[i]))
      return set_error(HE_ENOKEY, "rotation key " + std::to_string(pl.rot_keys[i]) + " not resident");
  return guarded([&] {
    Ev ev(h, s);
    he_ct y = conv_run(ev, *in, *in_map, out_ch, kernel, stride, padding, kernel_pts, mask_pts, out_map);
    ev.copy_out(y, out);
    if (bias_pt) ck(he_add_plain(h, out, bias_pt, out, s));  // the paper's "add the bias"
    return HE_OK;
  });
}

// the schedule options a layer's plan depends on, from its description
static int desc_options(const he_layer_desc* d, Ctx& opt) {
  if (d->log_n < 1 || d->log_n > 17) return set_error(HE_EINVAL, "log_n out of range");
  if (d->mask_chains != HE_CHAIN_HORNER && d->mask_chains != HE_CHAIN_BSGS)
    return set_error(HE_EINVAL, "unknown mask-chain mode");
  if (d->fc_form != HE_FC_ROWS && d->fc_form != HE_FC_DIAG) return set_error(HE_EINVAL, "unknown FC form");
  if (d->stride_mode != HE_STRIDE_EXTRACT && d->stride_mode != HE_STRIDE_LOG)
    return set_error(HE_EINVAL, "unknown striding mode");
  if (d->stride_groups != HE_STRIDE_JOINT && d->stride_groups != HE_STRIDE_GROUP_IN)
    return set_error(HE_EINVAL, "unknown stride grouping");
  if (d->channel_sum != HE_CHSUM_CHAIN && d->channel_sum != HE_CHSUM_LOG)
    return set_error(HE_EINVAL, "unknown channel-sum mode");
  opt.log_n = d->log_n;
  opt.n = 1 << d->log_n;
  opt.chain = d->mask_chains;
  opt.stride = d->stride_mode;
  opt.stride_groups = d->stride_groups;
  opt.chsum = d->channel_sum;
  opt.fc = d->fc_form;
  return HE_OK;
}

int he_layer_rotations(const he_layer_desc* d, he_layer_plan* plan) {
  if (!d || !plan) return set_error(HE_EINVAL, "null argument");
  return guarded([&] {
    Ctx opt;
    int rc = desc_options(d, opt);
    if (rc) return rc;
    switch (d->kind) {
      case HE_LAYER_CONV:
        return conv_plan(&opt, &d->in, d->out_ch, d->kernel, d->stride, d->padding, plan);
      case HE_LAYER_AVGPOOL:
        return pool_plan(&opt, &d->in, d->kernel, d->stride, plan);
      case HE_LAYER_FC:
        return fc_plan_impl(&opt, d->n_in, d->n_out, plan);
      case HE_LAYER_CHEB_MASK:
        *plan = he_layer_plan{};
        plan->n_mask_pts = 1;
        return HE_OK;
      default:
        return set_error(HE_EINVAL, "unknown layer kind");
    }
  });
}

int he_layer_plaintexts(const he_layer_desc* d, const double* weights, const double* bias, double* out,
                        size_t cap_vectors, int32_t* n_vectors) {
  if (!d || !n_vectors) return set_error(HE_EINVAL, "null argument");
  return guarded([&] {
    Ctx opt;  // the schedule options the layer's plan depends on
    int rc0 = desc_options(d, opt);
    if (rc0) return rc0;
    Vecs v;
    int rc;
    switch (d->kind) {
      case HE_LAYER_CONV:
        if (!weights) return set_error(HE_EINVAL, "convolution weights missing");
        rc = conv_vectors(&opt, d->in, d->out_ch, d->kernel, d->stride, d->padding, weights, bias, v);
        break;
      case HE_LAYER_AVGPOOL:
        rc = pool_vectors(&opt, d->in, d->kernel, d->stride, v);
        break;
      case HE_LAYER_FC:
        if (!weights) return set_error(HE_EINVAL, "fully connected weights missing");
        rc = fc_vectors(&opt, d->n_in, d->n_out, weights, bias, v);
        break;
      case HE_LAYER_CHEB_MASK: {
        if (!(d->beta > 0.0) || d->n_in < 0 || d->n_in > opt.n / 2) return set_error(HE_EINVAL, "bad scale mask");
        std::vector<double> m = zeros(opt.n / 2);
        for (int i = 0; i < d->n_in; i++) m[i] = 1.0 / d->beta;
        v.push_back(std::move(m));
        rc = HE_OK;
        break;
      }
      default:
        return set_error(HE_EINVAL, "unknown layer kind");
    }
    if (rc) return rc;
    *n_vectors = (int32_t)v.size();
    if (!out) return HE_OK;
    if (v.size() > cap_vectors) return set_error(HE_EINVAL, "output holds too few vectors");
    const size_t slots = (size_t)opt.n / 2;
    for (size_t i = 0; i < v.size(); i++) std::copy(v[i].begin(), v[i].end(), out + i * slots);
    return HE_OK;
  });
}

int he_avgpool_plan(const he_ctx* h, const he_fmap* in_map, int kernel, int stride, he_layer_plan* plan) {
  if (!h) return set_error(HE_EINVAL, "null context");
  return pool_plan(&h->c, in_map, kernel, stride, plan);
}

int he_avgpool(he_ctx* h, const he_ct* in, const he_fmap* in_map, int kernel, int stride, const he_pt* mask_pts,
               int n_mask_pts, he_ct* out, he_fmap* out_map, he_stream s) {
  if (!h || !out_map) return set_error(HE_EINVAL, "null argument");
  Ctx* c = &h->c;
  he_layer_plan pl;
  int rc;
  if ((rc = check_ct(c, in, "in"))) return rc;
  if ((rc = pool_plan(c, in_map, kernel, stride, &pl))) return rc;
  if (n_mask_pts != pl.n_mask_pts) return set_error(HE_EINVAL, "mask count differs from the layer plan");
  if (in->level <= pl.levels) return set_error(HE_ELEVEL, "not enough levels for the pooling");
  if ((rc = check_out(c, out, in->level - pl.levels))) return rc;
  if ((rc = check_pts(c, mask_pts, n_mask_pts, in->level, "mask_pts"))) return rc;
  for (int i = 0; i < pl.n_keys; i++)
    if (!key_known(c, pl.rot_keys[i]))
      return set_error(HE_ENOKEY, "rotation key " + std::to_string(pl.rot_keys[i]) + " not resident");
  return guarded([&] {
    Ev ev(h, s);
    he_ct y = pool_run(ev, *in, *in_map, kernel, stride, mask_pts, out_map);
    ev.copy_out(y, out);
    return HE_OK;
  });
}

int he_fc_plan(const he_ctx* h, int n_in, int n_out, he_layer_plan* plan) {
  if (!h) return set_error(HE_EINVAL, "null context");
  return fc_plan_impl(&h->c, n_in, n_out, plan);
}

int he_ctx_layer_streams(he_ctx* h, int n) {
  if (!h) return set_error(HE_EINVAL, "null context");
  if (n < 1 || n > 8) return set_error(HE_EINVAL, "layer streams must be in [1, 8]");
  h->c.layer_streams = n;
  return HE_OK;
}

int he_ctx_fc_form(he_ctx* h, int mode) {
  if (!h) return set_error(HE_EINVAL, "null context");
  if (mode != HE_FC_ROWS && mode != HE_FC_DIAG) return set_error(HE_EINVAL, "unknown fully connected form");
  h->c.fc = mode;
  return HE_OK;
}

int he_fc(he_ctx* h, const he_ct* in, int n_in, int n_out, const he_pt* weight_pts, const he_pt* mask_pts,
          const he_pt* bias_pt, he_ct* out, he_stream s) {
  if (!h) return set_error(HE_EINVAL, "null context");
  Ctx* c = &h->c;
  he_layer_plan pl;
  int rc;
  if ((rc = check_ct(c, in, "in"))) return rc;
  if ((rc = fc_plan_impl(c, n_in, n_out, &pl))) return rc;
  if (n_in > c->n / 2 || n_out > c->n / 2) return set_error(HE_EINVAL, "vector longer than the slots");
  if (in->level <= pl.levels) return set_error(HE_ELEVEL, "not enough levels for the fully connected layer");
  if ((rc = check_out(c, out, in->level - pl.levels))) return rc;
  if ((rc = check_pts(c, weight_pts, pl.n_kernel_pts, in->level, "weight_pts")) ||
      (pl.n_mask_pts && (rc = check_pts(c, mask_pts, 1, in->level - 1, "mask_pts"))))
    return rc;
  for (int i = 0; i < pl.n_keys; i++)
    if (!key_known(c, pl.rot_keys[i]))
      return set_error(HE_ENOKEY, "rotation key " + std::to_string(pl.rot_keys[i]) + " not resident");
  if (c->fc == HE_FC_DIAG && 2 * n_in > c->n / 2) return set_error(HE_EINVAL, "2 n_in exceeds the slots");
  return guarded([&] {
    Ev ev(h, s);
    if (c->fc == HE_FC_DIAG) {
      // x~ = x + Rot_{-n_in}(x); baby steps Rot_b(x~) hoisted; inner sums with
      // the pre-rotated diagonals; Horner over the giant steps with key B
      int B, A;
      bsgs_split(n_in, B, A);
      he_ct xt = ev.add_take(ev.rot(*in, -n_in), ev.copy(*in));
      std::vector<int> offs;
      for (int b = 1; b < B; b++) offs.push_back(b);
      std::vector<he_ct> baby{xt};
      if (!offs.empty())
        for (const he_ct& r : ev.rot_hoisted(xt, offs)) baby.push_back(r);
      auto inner = [&](int a) {
        const int cnt = std::min(B, n_in - a * B);
        std::vector<he_ct> cts(baby.begin(), baby.begin() + cnt);
        return mac_all(ev, cts, weight_pts + a * B);
      };
      he_ct acc = inner(A - 1);
      for (int a = A - 2; a >= 0; a--) acc = ev.add_take(ev.rot_take(acc, B), inner(a));
      for (const he_ct& b : baby) ev.release(b);
      acc = ev.rescale_take(acc);
      if (bias_pt) ck(he_add_plain(h, &acc, bias_pt, &acc, s));
      ev.copy_out(acc, out);
      return HE_OK;
    }
    auto neuron = [&](Ev& e, int k) {
      he_ct P = e.rescale_take(e.mul(*in, weight_pts[k]));
      for (int t = 1; t < n_in; t <<= 1) P = e.add_take(P, e.rot(P, t));
      he_ct r = e.rescale_take(e.mul(P, mask_pts[0]));
      e.release(P);
      return r;
    };
    he_ct acc{};
    {
      // neuron k on stream k mod K, then the placement chain on the caller's stream
      Fork fk(ev, std::min(c->streams_for_ring(), n_out));
      const int K = fk.size();
      if (K == 1) {
        acc = neuron(ev, n_out - 1);
        for (int k = n_out - 2; k >= 0; k--) acc = ev.add_take(ev.rot_take(acc, -1), neuron(ev, k));
      } else {
        std::vector<he_ct> r(n_out);
        for (int k = n_out - 1; k >= 0; k--) r[k] = neuron(fk.at(k % K), k);
        fk.join();
        acc = r[n_out - 1];  // rot_take returns only the caller evaluator's own temporaries
        for (int k = n_out - 2; k >= 0; k--) {
          acc = ev.rot_take(acc, -1);
          ev.add_into(acc, r[k]);
        }
      }
    }
    if (bias_pt) ck(he_add_plain(h, &acc, bias_pt, &acc, s));
    ev.copy_out(acc, out);
    return HE_OK;
  });
}

int he_poly4(he_ctx* h, const he_ct* in, const double* cf, double delta, he_ct* out, he_stream s) {
  if (!h || !cf) return set_error(HE_EINVAL, "null argument");
  Ctx* c = &h->c;
  int rc;
  if ((rc = check_ct(c, in, "in"))) return rc;
  if (cf[3] != 0.0) return set_error(HE_EUNSUPPORTED, "the cubic coefficient must be zero");
  if (in->level <= 3) return set_error(HE_ELEVEL, "the polynomial needs three levels");
  if ((rc = check_out(c, out, in->level - 3))) return rc;
  if (!key_known(c, HE_KEY_RELIN)) return set_error(HE_ENOKEY, "relinearization key not resident");
  return guarded([&] {
    Ev ev(h, s);
    const he_ct& x = *in;
    he_ct x2 = ev.rescale(ev.mul_relin(x, x));
    he_ct t = ev.add_const(ev.rescale(ev.mul_const(x2, cf[4], delta)), cf[2]);
    he_ct v = ev.rescale(ev.mul_relin(Ev::drop(x2, t.level), t));
    const double q = (double)c->mod[v.level];
    const double sigma = v.scale * q / x.scale;
    he_ct lin = ev.rescale(ev.mul_const(Ev::drop(x, v.level + 1), cf[1], sigma));
    lin.scale = v.scale;
    he_ct p = ev.add_const(ev.add(v, lin), cf[0]);
    ev.copy_out(p, out);
    return HE_OK;
  });
}

int he_cheb_relu_coeffs(double beta, int degree, double* cf) {
  if (!cf || degree < 1 || degree > HE_CHEB_MAX_DEGREE || !(beta > 0.0))
    return set_error(HE_EINVAL, "need beta > 0 and degree in [1, 255]");
  const int n = degree + 1;
  const double pi = 3.14159265358979323846;
  for (int j = 0; j < n; j++) {
    double acc = 0.0;
    for (int k = 0; k < n; k++) {
      const double th = pi * (k + 0.5) / n;
      acc += beta * std::max(0.0, std::cos(th)) * std::cos(j * th);
    }
    cf[j] = 2.0 / n * acc;
  }
  // f = beta z / 2 + beta |z| / 2: the odd part is exactly beta T_1 / 2
  for (int j = 1; j < n; j += 2) cf[j] = 0.0;
  cf[1] = beta / 2.0;
  return HE_OK;
}

int he_cheb_plan(const double* coeffs, int degree, int masked, int32_t* levels, int32_t* relins) {
  if (!levels || !relins) return set_error(HE_EINVAL, "null argument");
  int l = 0, r = 0;
  int rc = cheb_plan_impl(coeffs, degree, masked, &l, &r);
  if (rc) return rc;
  *levels = l;
  *relins = r;
  return HE_OK;
}

int he_cheb(he_ctx* h, const he_ct* in, const he_pt* scale_mask, const double* cf, int degree, double delta,
            he_ct* out, he_stream s) {
  if (!h || !cf) return set_error(HE_EINVAL, "null argument");
  Ctx* c = &h->c;
  int rc, levels = 0, relins = 0;
  if ((rc = check_ct(c, in, "in"))) return rc;
  if ((rc = cheb_plan_impl(cf, degree, scale_mask != nullptr, &levels, &relins))) return rc;
  if (in->level <= levels)
    return set_error(HE_ELEVEL, "the Chebyshev evaluation needs " + std::to_string(levels) + " levels");
  if (scale_mask && (rc = check_pts(c, scale_mask, 1, in->level, "scale_mask"))) return rc;
  if ((rc = check_out(c, out, in->level - levels))) return rc;
  if (!key_known(c, HE_KEY_RELIN)) return set_error(HE_ENOKEY, "relinearization key not resident");
  const std::vector<ChebNode> tree = cheb_tree(cf, degree);
  const std::vector<int> terms = cheb_terms(tree);
  return guarded([&] {
    Ev ev(h, s);
    const he_ct v = scale_mask ? ev.rescale_take(ev.mul(*in, *scale_mask)) : *in;
    // the terms on up to two streams (the caller's and a helper), each placed
    // by list scheduling (one unit per product, earliest start, ties to a
    // factor's stream); a term waits for a factor made on the other stream.
    // The division tree's remainder branch at the root then runs on the
    // helper beside the quotient branch.  Every value is computed by the same
    // operations as on one stream.
    Fork fk(ev, std::min(c->streams_for_ring(), 2));
    const int K = fk.size();
    auto stream_of = [&](int k) { return (hipStream_t)fk.at(k).s; };
    std::vector<he_ct> T(degree + 1);
    std::vector<int> on(degree + 1, 0), fin(degree + 1, 0), busy(K, 0);
    T[1] = v;
    for (size_t t = 1; t < terms.size(); t++) {
      const int j = terms[t];
      const int a = j / 2, b = j - j / 2;
      const int dep = std::max(fin[a], fin[b]);
      int k = on[b];
      for (int x = 0; x < K; x++)
        if (std::max(dep, busy[x]) < std::max(dep, busy[k])) k = x;
      hipStream_t to = stream_of(k);
      for (int f : {a, b})
        if (on[f] != k) ck(stream_fork(stream_of(on[f]), &to, 1));
      Ev& e = fk.at(k);
      const int lv = std::min(T[a].level, T[b].level);
      he_ct p = e.rescale_take(e.mul_relin(Ev::drop(T[a], lv), Ev::drop(T[b], lv)));
      he_ct p2 = e.add(p, p);
      e.release(p);
      if (j % 2 == 0) {
        T[j] = e.add_const(p2, -1.0);
      } else {
        he_ct l = cheb_lift(e, v, p2.level, p2.scale, -1.0);
        T[j] = e.add(p2, l);
        e.release(l);
      }
      e.release(p2);
      on[j] = k;
      fin[j] = std::max(dep, busy[k]) + 1;
      busy[k] = fin[j];
    }
    const int top = v.level + cheb_allowed(tree, 0, 0);
    he_ct y{};
    if (K > 1 && tree[0].K) {
      // both streams see every term; remainder r' on the helper, quotient
      // branch and the root product on the caller's stream
      const ChebNode& n = tree[0];
      fk.join();
      hipStream_t helper = stream_of(1);
      ck(stream_fork(stream_of(0), &helper, 1));
      he_ct rc = cheb_eval_node(fk.at(1), tree, n.r, T, top, delta);
      const double sigma = delta * (double)c->mod[top] / T[n.K].scale;
      he_ct qc = cheb_eval_node(ev, tree, n.q, T, top + 1, sigma);
      he_ct p = ev.rescale_take(ev.mul_relin(qc, Ev::drop(T[n.K], top + 1)));
      ev.release(qc);
      p.scale = delta;
      fk.join();
      y = ev.add_take(p, rc);
    } else {
      fk.join();
      y = cheb_eval_node(ev, tree, 0, T, top, delta);
    }
    ev.copy_out(y, out);
    return HE_OK;
  });
}

}  // extern "C"

// ---------------------------------------------------------------- bootstrapping
// The standard four-stage RNS-CKKS bootstrapping (ModRaise, CoeffToSlot,
// EvalMod, SlotToCoeff) composed of the calls above; every choice is the
// one he.h documents (plan, scales, rescale placement), so that the
// composition is bit-exact against a CPU definition of the same steps.
namespace he {

// stages per level: as even as possible, larger groups first
static std::vector<int> boot_group_sizes(int total, int levels) {
  std::vector<int> g(levels, total / levels);
  for (int i = 0; i < total % levels; i++) g[i]++;
  return g;
}

// block half-sizes h of each level in application order: CoeffToSlot runs
// the inverse stages h = n/2 .. 1, SlotToCoeff the forward ones h = 1 .. n/2
// (CoeffToSlot's groups mirrored)
static std::vector<std::vector<int>> boot_groups(int log_slots, int levels, bool inverse) {
  std::vector<std::vector<int>> out;
  int at = log_slots - 1;
  for (int sz : boot_group_sizes(log_slots, levels)) {
    std::vector<int> hs;
    for (int t = 0; t < sz; t++) hs.push_back(1 << at--);
    out.push_back(hs);
  }
  if (!inverse) {
    std::reverse(out.begin(), out.end());
    for (auto& g : out) std::reverse(g.begin(), g.end());
  }
  return out;
}

static long long floor_div(long long a, long long b) { return a / b - ((a % b != 0) && ((a < 0) != (b < 0))); }

// Baby-step giant-step layout of one level: shifts d = u k (k centred mod
// n/u), k = i + B j, B the smallest power of two with B^2 >= span.
struct BootLevel {
  int n = 0, u = 1, B = 1;
  std::vector<int> babies;  // i > 0 used, ascending
  std::vector<std::pair<int, std::vector<std::pair<int, int>>>> giants;  // j ascending: (i, shift mod n)
  int count() const {
    int c = 0;
    for (auto& g : giants) c += (int)g.second.size();
    return c;
  }
  int baby_rot(int i) const { return (int)(((long long)u * i) % n); }
  int giant_rot(int j) const {
    long long r = ((long long)u * B * j) % n;
    return (int)(r < 0 ? r + n : r);
  }
};

// the level's shifts: every sum of +-h or 0 over its stages (mod n), which
// is where the product of the butterfly stages has nonzero diagonals
static BootLevel boot_level(int n, const std::vector<int>& hs) {
  std::vector<char> have(n, 0), next(n, 0);
  have[0] = 1;
  for (int h : hs) {
    std::fill(next.begin(), next.end(), 0);
    for (int d = 0; d < n; d++)
      if (have[d]) {
        next[d] = 1;
        next[(d + h) % n] = 1;
        next[((d - h) % n + n) % n] = 1;
      }
    have.swap(next);
  }
  BootLevel p;
  p.n = n;
  p.u = *std::min_element(hs.begin(), hs.end());
  const int m = n / p.u;
  std::vector<int> ks;
  for (int d = 0; d < n; d++)
    if (have[d]) {
      int k = (d / p.u) % m;
      if (k > m / 2) k -= m;
      ks.push_back(k);
    }
  std::sort(ks.begin(), ks.end());
  const int span = ks.back() - ks.front() + 1;
  while (p.B * p.B < span) p.B *= 2;
  std::map<int, std::vector<std::pair<int, int>>> by_j;
  for (int k : ks) {
    const int j = (int)floor_div(k, p.B), i = k - p.B * j;
    by_j[j].push_back({i, (int)((((long long)p.u * k) % n + n) % n)});
  }
  std::vector<char> used(p.B, 0);
  for (auto& kv : by_j) {
    std::sort(kv.second.begin(), kv.second.end());
    for (auto& t : kv.second) used[t.first] = 1;
    p.giants.push_back(kv);
  }
  for (int i = 1; i < p.B; i++)
    if (used[i]) p.babies.push_back(i);
  return p;
}

struct BootPlanC {
  int n = 0;
  std::vector<std::vector<int>> cts_hs, stc_hs;
  std::vector<BootLevel> cts, stc;
};

static int boot_plan_build(int log_n, int levels, BootPlanC* out) {
  const int ls = log_n - 1;
  out->n = 1 << ls;
  out->cts_hs = boot_groups(ls, levels, true);
  out->stc_hs = boot_groups(ls, levels, false);
  out->cts.clear();
  out->stc.clear();
  for (auto& hs : out->cts_hs) out->cts.push_back(boot_level(out->n, hs));
  for (auto& hs : out->stc_hs) out->stc.push_back(boot_level(out->n, hs));
  return HE_OK;
}

// The plan depends only on (log_n, levels): built once per process and
// copied out (the shift sets take a few hundred microseconds at N = 2^16).
static int boot_plan_make(int log_n, int levels, BootPlanC* out) {
  if (log_n < 2 || log_n > 16) return set_error(HE_EINVAL, "ring degree out of range");
  if (levels < 1 || levels > log_n - 1) return set_error(HE_EINVAL, "transform levels out of range");
  static std::mutex mu;
  static std::map<std::pair<int, int>, BootPlanC> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find({log_n, levels});
  if (it == cache.end()) {
    BootPlanC p;
    int rc;
    if ((rc = boot_plan_build(log_n, levels, &p))) return rc;
    it = cache.emplace(std::make_pair(log_n, levels), std::move(p)).first;
  }
  *out = it->second;
  return HE_OK;
}

// diagonals of one butterfly stage / of a product of diagonal matrices
using Cd = std::complex<double>;
using Diags = std::map<int, std::vector<Cd>>;

static Cd slot_root(int m, int j) {
  uint64_t e = 1;
  for (int t = 0; t < j; t++) e = e * 5 % (4 * (uint64_t)m);
  return std::polar(1.0, 2.0 * M_PI * (double)e / (4.0 * m));
}

static void diag_put(Diags& d, int shift, const std::vector<Cd>& v) {
  auto it = d.find(shift);
  if (it == d.end()) {
    d[shift] = v;
  } else {
    for (size_t p = 0; p < v.size(); p++) it->second[p] += v[p];
  }
}

static Diags stage_diags(int n, int h, bool inverse) {
  std::vector<Cd> roots(h);
  for (int j = 0; j < h; j++) roots[j] = slot_root(2 * h, j);
  std::vector<Cd> d0(n), dp(n), dm(n);
  for (int p = 0; p < n; p++) {
    const int r = p % (2 * h);
    const bool first = r < h;
    const Cd x = roots[first ? r : r - h];
    if (inverse) {
      d0[p] = first ? Cd(0.5, 0.0) : -0.5 / x;
      dp[p] = first ? Cd(0.5, 0.0) : Cd(0.0, 0.0);
      dm[p] = first ? Cd(0.0, 0.0) : 0.5 / x;
    } else {
      d0[p] = first ? Cd(1.0, 0.0) : -x;
      dp[p] = first ? x : Cd(0.0, 0.0);
      dm[p] = first ? Cd(0.0, 0.0) : Cd(1.0, 0.0);
    }
  }
  Diags out;
  out[0] = d0;
  diag_put(out, h % n, dp);
  diag_put(out, ((-h) % n + n) % n, dm);
  return out;
}

// A B (B applied first): C_{d+e}[p] += A_d[p] B_e[(p + d) mod n]
static Diags diag_compose(const Diags& a, const Diags& b, int n) {
  Diags out;
  std::vector<Cd> t(n);
  for (auto& da : a)
    for (auto& db : b) {
      for (int p = 0; p < n; p++) t[p] = da.second[p] * db.second[(p + da.first) % n];
      diag_put(out, (da.first + db.first) % n, t);
    }
  return out;
}

// CoeffToSlot's EvalMod range K and raise exponent e for a context
static void boot_raise(const Ctx* c, const he_boot_desc* d, int* e, double* K, double* raise) {
  const double q0 = (double)c->mod[0];
  const double bound = 2.0 * q0 * d->k_min;
  int x = 0;
  while (std::ldexp(d->delta, x) < bound) x++;
  *e = x;
  *raise = std::ldexp(d->delta, x);
  *K = *raise / (2.0 * q0);
}

static void boot_mod_coeffs_impl(double K, int degree, int r, double* cf) {
  const int n = degree + 1;
  std::vector<double> th(n), fx(n);
  for (int k = 0; k < n; k++) {
    th[k] = M_PI * (k + 0.5) / n;
    fx[k] = r ? std::cos(2.0 * M_PI * (K * std::cos(th[k]) - 0.25) / (double)(1 << r))
              : std::sin(2.0 * M_PI * K * std::cos(th[k])) / (2.0 * M_PI);
  }
  for (int j = 0; j < n; j++) {
    double s = 0.0;
    for (int k = 0; k < n; k++) s += fx[k] * std::cos(j * th[k]);
    cf[j] = (r == 0 && j % 2 == 0) ? 0.0 : 2.0 / n * s;
  }
}

// levels, plaintext scales and the Chebyshev level count for a context
struct BootScales {
  int level_in = 0, cheb_levels = 0, cheb_relins = 0, e = 0;
  double K = 0, raise = 0;
  std::vector<double> cts, stc;
};

static int boot_scales_impl(const Ctx* c, const he_boot_desc* d, BootScales* s) {
  if (!d) return set_error(HE_EINVAL, "null description");
  if (d->levels < 1 || d->levels > c->log_n - 1) return set_error(HE_EINVAL, "transform levels out of range");
  if (d->degree < 1 || d->degree > HE_CHEB_MAX_DEGREE) return set_error(HE_EINVAL, "EvalMod degree out of range");
  if (!(d->k_min > 0.0) || !(d->delta > 1.0)) return set_error(HE_EINVAL, "k_min and delta must be positive");
  if (d->double_angles < 0 || d->double_angles > 8) return set_error(HE_EINVAL, "double angles out of range");
  s->level_in = d->level ? d->level : c->L;
  if (s->level_in < 1 || s->level_in > c->L) return set_error(HE_ELEVEL, "raise level out of range");
  boot_raise(c, d, &s->e, &s->K, &s->raise);
  std::vector<double> cf(d->degree + 1);
  boot_mod_coeffs_impl(s->K, d->degree, d->double_angles, cf.data());
  int rc;
  if ((rc = cheb_plan_impl(cf.data(), d->degree, 0, &s->cheb_levels, &s->cheb_relins))) return rc;
  s->cheb_levels += d->double_angles;  // EvalMod's levels
  const int out_level = s->level_in - 2 * d->levels - s->cheb_levels;
  if (out_level < 1)
    return set_error(HE_ELEVEL, "bootstrapping needs " + std::to_string(2 * d->levels + s->cheb_levels + 1) +
                                    " levels");
  const std::vector<int> ex = boot_group_sizes(s->e, d->levels);
  const double a = d->double_angles ? 2.0 * M_PI : 1.0;
  const double f2 = std::log2((double)c->mod[0] / (d->delta * a));
  const int f = (int)std::floor(f2 + 0.5);
  const std::vector<int> fx = f > 0 ? boot_group_sizes(f, d->levels) : std::vector<int>(d->levels, 0);
  s->cts.resize(d->levels);
  s->stc.resize(d->levels);
  for (int g = 0; g < d->levels; g++) {
    s->cts[g] = std::ldexp((double)c->mod[s->level_in - g - 1], -ex[g]);
    const int l = s->level_in - d->levels - s->cheb_levels - g;
    s->stc[g] = std::ldexp((double)c->mod[l - 1], fx[g]);
  }
  return HE_OK;
}

// y = sum_d D_d (.) Rot_d(x) by baby-step giant-step (pts in consumption
// order).  The giant steps (each a product-sum, a rescale and a rotation)
// are independent: they are dealt round-robin to `streams` streams, each
// keeping its own partial sum; the partial sums are added on the caller's
// stream.  Modular additions commute, so the result does not depend on the
// split.
static he_ct boot_transform(Ev& ev, const he_ct& x, const BootLevel& p, const he_pt* pts, int streams) {
  std::vector<int> rots;
  for (int i : p.babies) rots.push_back(p.baby_rot(i));
  std::vector<he_ct> br = ev.rot_hoisted(x, rots);
  std::vector<he_ct> baby(p.B);
  baby[0] = x;
  for (size_t t = 0; t < p.babies.size(); t++) baby[p.babies[t]] = br[t];
  he_ct acc{};
  {
    Fork fk(ev, std::min(streams, (int)p.giants.size()));
    const int K = fk.size();
    std::vector<he_ct> part(K);
    std::vector<char> have(K, 0);
    int t = 0;
    for (size_t gi = 0; gi < p.giants.size(); gi++) {
      const auto& g = p.giants[gi];
      const int k = (int)(gi % K);
      Ev& e = fk.at(k);
      std::vector<he_ct> terms;
      for (auto& iq : g.second) terms.push_back(baby[iq.first]);
      he_ct s = mac_all(e, terms, pts + t);
      t += (int)g.second.size();
      s = e.rescale_take(s);
      if (g.first != 0) s = e.rot_take(s, p.giant_rot(g.first));
      if (!have[k]) {
        part[k] = s;
        have[k] = 1;
      } else {
        part[k] = e.add_take(part[k], s);
      }
    }
    fk.join();
    acc = part[0];  // on the caller's stream (k = 0 is the caller's evaluator)
    for (int k = 1; k < K; k++)
      if (have[k]) ck(he_add(ev.h, &acc, &part[k], &acc, ev.s));
  }
  for (auto& b : br) ev.release(b);
  return acc;
}

}  // namespace he

extern "C" {

int he_boot_plan(int32_t log_n, int32_t levels, int32_t* rotations, int32_t* n_rotations, int32_t* counts,
                 int32_t* n_key_switches) {
  if (!rotations || !n_rotations || !counts) return set_error(HE_EINVAL, "null argument");
  BootPlanC p;
  int rc;
  if ((rc = boot_plan_make(log_n, levels, &p))) return rc;
  std::vector<int> r;
  int ks = 0;
  for (const auto* side : {&p.cts, &p.stc})
    for (const BootLevel& lv : *side) {
      for (int i : lv.babies) r.push_back(lv.baby_rot(i)), ks += lv.baby_rot(i) != 0;
      for (auto& g : lv.giants)
        if (g.first != 0) r.push_back(lv.giant_rot(g.first)), ks += lv.giant_rot(g.first) != 0;
    }
  if (n_key_switches) *n_key_switches = ks;
  std::sort(r.begin(), r.end());
  r.erase(std::unique(r.begin(), r.end()), r.end());
  r.erase(std::remove(r.begin(), r.end(), 0), r.end());
  if ((int)r.size() > HE_BOOT_MAX_ROTATIONS) return set_error(HE_EUNSUPPORTED, "too many rotation keys");
  for (size_t i = 0; i < r.size(); i++) rotations[i] = r[i];
  *n_rotations = (int32_t)r.size();
  for (int g = 0; g < levels; g++) {
    counts[g] = p.cts[g].count();
    counts[levels + g] = p.stc[g].count();
  }
  return HE_OK;
}

int he_boot_diagonals(int32_t log_n, int32_t levels, int32_t inverse, double* re, double* im, size_t cap) {
  if (!re || !im) return set_error(HE_EINVAL, "null argument");
  BootPlanC p;
  int rc;
  if ((rc = boot_plan_make(log_n, levels, &p))) return rc;
  const int n = p.n;
  const auto& hs_all = inverse ? p.cts_hs : p.stc_hs;
  const auto& plans = inverse ? p.cts : p.stc;
  size_t total = 0;
  for (auto& lv : plans) total += (size_t)lv.count() * n;
  if (cap < total) return set_error(HE_EINVAL, "output too small for the diagonals");
  try {
    size_t at = 0;
    for (size_t g = 0; g < plans.size(); g++) {
      Diags m;
      m[0] = std::vector<Cd>(n, Cd(1.0, 0.0));
      for (int h : hs_all[g]) m = diag_compose(stage_diags(n, h, inverse != 0), m, n);
      const BootLevel& lv = plans[g];
      for (auto& gj : lv.giants) {
        const long long sh = (long long)lv.u * lv.B * gj.first;  // pre-rotation: D[p - u B j]
        for (auto& t : gj.second) {
          auto it = m.find(t.second);
          for (int q = 0; q < n; q++) {
            Cd v(0.0, 0.0);
            if (it != m.end()) v = it->second[(size_t)((((q - sh) % n) + n) % n)];
            re[at + q] = v.real();
            im[at + q] = v.imag();
          }
          at += n;
        }
      }
    }
  } catch (const std::bad_alloc&) {
    return set_error(HE_ENOMEM, "host allocation failed");
  }
  return HE_OK;
}

int he_boot_mod_coeffs(double K, int32_t degree, int32_t double_angles, double* coeffs) {
  if (!coeffs) return set_error(HE_EINVAL, "null argument");
  if (degree < 1 || degree > HE_CHEB_MAX_DEGREE) return set_error(HE_EINVAL, "degree out of range");
  if (!(K > 0.0)) return set_error(HE_EINVAL, "K must be positive");
  if (double_angles < 0 || double_angles > 8) return set_error(HE_EINVAL, "double angles out of range");
  boot_mod_coeffs_impl(K, degree, double_angles, coeffs);
  return HE_OK;
}

int he_boot_scales(const he_ctx* h, const he_boot_desc* desc, double* K, double* raise_scale, double* cts_scales,
                   double* stc_scales) {
  if (!h || !K || !raise_scale || !cts_scales || !stc_scales) return set_error(HE_EINVAL, "null argument");
  BootScales s;
  int rc;
  if ((rc = boot_scales_impl(&h->c, desc, &s))) return rc;
  *K = s.K;
  *raise_scale = s.raise;
  for (int g = 0; g < desc->levels; g++) {
    cts_scales[g] = s.cts[g];
    stc_scales[g] = s.stc[g];
  }
  return HE_OK;
}

int he_bootstrap(he_ctx* h, const he_ct* in, const he_boot_desc* desc, const he_pt* cts_pts, const he_pt* stc_pts,
                 const double* coeffs, he_ct* out, he_stream s) {
  if (!h || !coeffs) return set_error(HE_EINVAL, "null argument");
  Ctx* c = &h->c;
  int rc;
  if ((rc = check_ct(c, in, "in"))) return rc;
  // Capture of a bootstrap is verified at N = 2^12 only: at N = 2^16 (where
  // the Chebyshev evaluation forks helper streams of the helper stream it
  // runs on) a captured bootstrap ended the process once, cause not found.
  if (c->n >= 65536 && stream_capturing((hipStream_t)s))
    return set_error(HE_EUNSUPPORTED, "bootstrapping cannot be captured into a graph at N >= 2^16");
  BootScales sc;
  if ((rc = boot_scales_impl(c, desc, &sc))) return rc;
  BootPlanC p;
  if ((rc = boot_plan_make(c->log_n, desc->levels, &p))) return rc;
  const int levels = desc->levels;
  const int out_level = sc.level_in - 2 * levels - sc.cheb_levels;
  if ((rc = check_out(c, out, out_level))) return rc;
  if (out->data == in->data) return set_error(HE_EINVAL, "bootstrapping output aliases the input");
  // plaintexts: CoeffToSlot level g at level_in - g, SlotToCoeff level g at
  // the level it is applied at
  {
    int at = 0;
    for (int g = 0; g < levels; g++) {
      if ((rc = check_pts(c, cts_pts ? cts_pts + at : nullptr, p.cts[g].count(), sc.level_in - g, "cts_pts")))
        return rc;
      at += p.cts[g].count();
    }
    at = 0;
    for (int g = 0; g < levels; g++) {
      const int l = sc.level_in - levels - sc.cheb_levels - g;
      if ((rc = check_pts(c, stc_pts ? stc_pts + at : nullptr, p.stc[g].count(), l, "stc_pts"))) return rc;
      at += p.stc[g].count();
    }
  }
  for (const auto* side : {&p.cts, &p.stc})
    for (const BootLevel& lv : *side) {
      for (int i : lv.babies)
        if (lv.baby_rot(i) != 0 && !key_known(c, lv.baby_rot(i)))
          return set_error(HE_ENOKEY, "bootstrapping rotation key missing");
      for (auto& g : lv.giants)
        if (g.first != 0 && lv.giant_rot(g.first) != 0 && !key_known(c, lv.giant_rot(g.first)))
          return set_error(HE_ENOKEY, "bootstrapping rotation key missing");
    }
  if (!key_known(c, HE_KEY_CONJ)) return set_error(HE_ENOKEY, "conjugation key not resident");
  if (!key_known(c, HE_KEY_RELIN)) return set_error(HE_ENOKEY, "relinearization key not resident");
  const double q0 = (double)c->mod[0];
  const double in_scale = in->scale;
  return guarded([&] {
    Ev ev(h, s);
    const he_ct in1{in->data, 1, in->cap, in->scale};
    he_ct x = ev.fresh();
    ck(he_mod_raise(h, &in1, sc.level_in, &x, s));
    x.scale = sc.raise;
    const int streams = std::max(1, c->layer_streams);
    int at = 0;
    for (int g = 0; g < levels; g++) {
      he_ct y = boot_transform(ev, x, p.cts[g], cts_pts + at, streams);
      at += p.cts[g].count();
      ev.release(x);
      x = y;
    }
    // EvalMod on the real and imaginary parts
    he_ct w = ev.rot(x, HE_KEY_CONJ);
    he_ct re = ev.add(x, w);
    he_ct df = ev.fresh();
    ck(he_sub(h, &x, &w, &df, s));
    ev.release(w);
    ev.release(x);
    he_ct im = ev.fresh();
    ck(he_mul_i(h, &df, -1, &im, s));
    ev.release(df);
    he_ct re2 = ev.fresh(), im2 = ev.fresh();
    {
      // the two parts on two streams when helpers are allowed; each part's
      // last step writes its result into a buffer of the caller's evaluator.
      // Where the Chebyshev evaluation itself forks (N = 2^16), the caller's
      // part borrows the caller's first helper, so the other part takes a
      // second one: the parts then overlap, and no helper's temporaries are
      // handed from one part to the other.
      Fork fk(ev, c->streams_for_ring() > 1 ? 3 : std::min(streams, 2));
      auto evalmod = [&](Ev& e, const he_ct& part, he_ct& res) {
        const int r = desc->double_angles;
        if (r == 0) {
          ck(he_cheb(h, &part, nullptr, coeffs, desc->degree, desc->delta, &res, e.s));
          return;
        }
        he_ct c0 = e.fresh();
        ck(he_cheb(h, &part, nullptr, coeffs, desc->degree, desc->delta, &c0, e.s));
        for (int t = 0; t < r; t++) {
          he_ct p2 = e.rescale_take(e.mul_relin(c0, c0));
          e.release(c0);
          he_ct sum = e.add(p2, p2);
          e.release(p2);
          if (t + 1 < r) {
            c0 = e.add_const(sum, -1.0);
          } else {
            ck(he_add_const(h, &sum, -1.0, &res, e.s));
          }
          e.release(sum);
        }
        res.scale = res.scale * (2.0 * M_PI);
      };
      evalmod(ev, re, re2);
      evalmod(fk.at(fk.size() - 1), im, im2);
      fk.join();
    }
    ev.release(re);
    ev.release(im);
    ck(he_mul_i(h, &im2, 1, &im2, s));
    he_ct z = ev.add_take(re2, im2);
    at = 0;
    for (int g = 0; g < levels; g++) {
      he_ct y = boot_transform(ev, z, p.stc[g], stc_pts + at, streams);
      at += p.stc[g].count();
      ev.release(z);
      z = y;
    }
    ev.copy_out(z, out);
    out->scale = z.scale * (in_scale / q0);
    return HE_OK;
  });
}

}  // extern "C"
