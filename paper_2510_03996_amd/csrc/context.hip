// Context creation: prime chain, NTT twiddles, basis-conversion constants,
// resident key store and the workspace pool.
#include <algorithm>
#include <cstring>
#include <string>

#include "internal.h"

namespace he {

static thread_local std::string g_err;

int set_error(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
int hip_error(hipError_t e, const char* what) {
  return set_error(HE_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------- host modular helpers
typedef unsigned __int128 u128;
static uint64_t hmul(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }
static uint64_t hpow(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  a %= q;
  for (; e; e >>= 1) {
    if (e & 1) r = hmul(r, a, q);
    a = hmul(a, a, q);
  }
  return r;
}
static uint64_t hinv(uint64_t a, uint64_t q) { return hpow(a, q - 2, q); }
static uint64_t shoup_of(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }

static bool miller_rabin(uint64_t n) {
  if (n < 2) return false;
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (uint64_t b : bases) {
    if (n % b == 0) return n == b;
  }
  uint64_t d = n - 1;
  int s = 0;
  while (!(d & 1)) { d >>= 1; s++; }
  for (uint64_t b : bases) {
    uint64_t x = hpow(b, d, n);
    if (x == 1 || x == n - 1) continue;
    bool composite = true;
    for (int r = 1; r < s; r++) {
      x = hmul(x, x, n);
      if (x == n - 1) { composite = false; break; }
    }
    if (composite) return false;
  }
  return true;
}

static int brv(int x, int logn) {
  int r = 0;
  for (int i = 0; i < logn; i++) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
}

// minimum primitive 2N-th root of unity mod q
static uint64_t min_psi(uint64_t q, uint64_t n) {
  uint64_t cand = 0;
  for (uint64_t x = 2;; x++) {
    cand = hpow(x, (q - 1) / (2 * n), q);
    if (hpow(cand, n, q) == q - 1) break;
  }
  uint64_t sq = hmul(cand, cand, q), cur = cand, best = cand;
  for (uint64_t t = 1; t < n; t++) {
    cur = hmul(cur, sq, q);
    if (cur < best) best = cur;
  }
  return best;
}

LimbMap range_map(int first_pos, int n, int first_mod) {
  LimbMap m{};
  m.n = n;
  for (int i = 0; i < n; i++) {
    m.pos[i] = (uint16_t)(first_pos + i);
    m.mod[i] = (uint8_t)(first_mod + i);
  }
  return m;
}

LimbMap ext_map(const Ctx* c, int level) {
  LimbMap m{};
  m.n = level + c->K;
  for (int i = 0; i < m.n; i++) {
    m.pos[i] = (uint16_t)i;
    m.mod[i] = (uint8_t)(i < level ? i : c->L + (i - level));
  }
  return m;
}

int32_t norm_key_id(const Ctx* c, int32_t id) {
  if (id == HE_KEY_RELIN || id == HE_KEY_CONJ) return id;
  int32_t h = c->n / 2;
  int32_t r = id % h;
  return r < 0 ? r + h : r;
}

uint32_t galois_elt(const Ctx* c, int32_t r) {
  uint64_t two_n = 2 * (uint64_t)c->n;
  if (r == HE_KEY_CONJ) return (uint32_t)(two_n - 1);
  return (uint32_t)hpow(5, (uint64_t)norm_key_id(c, r), two_n);
}

uint64_t omega4(const Ctx* c, int m) { return hpow(c->psi[m], (uint64_t)c->n / 2, c->mod[m]); }

template <class T>
static int dev_alloc(Ctx* c, T** p, size_t count) {
  void* v = nullptr;
  hipError_t e = hipMalloc(&v, count * sizeof(T));
  if (e != hipSuccess) return set_error(HE_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  c->allocs.push_back(v);
  *p = (T*)v;
  return HE_OK;
}

// Host-side construction of one basis-conversion descriptor (constants are
// uploaded to device memory; the descriptor points at them).
static int build_conv(Ctx* c, ConvDesc& t, const std::vector<int>& in_pos, const std::vector<int>& in_mod,
                      const std::vector<int>& out_pos, const std::vector<int>& out_mod) {
  t = ConvDesc{};
  t.nin = (int)in_mod.size();
  t.nout = (int)out_mod.size();
  if (t.nin > MAX_BCONV_IN || t.nout > MAX_BCONV_OUT) return set_error(HE_EINVAL, "basis conversion too wide");
  for (int i = 0; i < t.nin; i++) { t.in_pos[i] = in_pos[i]; t.in_mod[i] = in_mod[i]; }
  // outputs of 51 bits and more (integer arithmetic) first, then the FP64 ones
  t.nint = 0;
  {
    int n = 0;
    for (int pass = 0; pass < 2; pass++)
      for (size_t p = 0; p < out_mod.size(); p++)
        if (conv_out_f64(c->hmod[out_mod[p]].k) == (pass == 1)) {
          t.out_pos[n] = out_pos[p];
          t.out_mod[n] = out_mod[p];
          n++;
          if (pass == 0) t.nint++;
        }
  }
  // parts: one per narrow input, two (low 32 bits, the rest) per wide one
  std::vector<int> part_in, part_sh;
  for (int i = 0; i < t.nin; i++) {
    if (conv_in_narrow(c->hmod[in_mod[i]].k)) {
      t.part_pos[part_in.size()] = in_pos[i];
      t.part_kind[part_in.size()] = 0;
      part_in.push_back(i);
      part_sh.push_back(0);
    } else {
      for (int h = 0; h < 2; h++) {
        t.part_pos[part_in.size()] = in_pos[i];
        t.part_kind[part_in.size()] = 1 + h;
        part_in.push_back(i);
        part_sh.push_back(32 * h);
      }
    }
  }
  t.nparts = (int)part_in.size();
  std::vector<uint64_t> cst((size_t)t.nout * t.nparts * 2, 0);
  for (int p = 0; p < t.nout; p++) {
    const uint64_t po = c->mod[t.out_mod[p]];
    const bool f64 = conv_out_f64(c->hmod[t.out_mod[p]].k);
    for (int v = 0; v < t.nparts; v++) {
      // [Qin / q_i]_p 2^shift for the part's input i
      const int i = part_in[v];
      uint64_t w = 1 % po;
      for (int i2 = 0; i2 < t.nin; i2++)
        if (i2 != i) w = hmul(w, c->mod[in_mod[i2]] % po, po);
      w = hmul(w, (uint64_t)(((u128)1 << part_sh[v]) % po), po);
      uint64_t* e = &cst[((size_t)p * t.nparts + v) * 2];
      if (f64) {
        const double wc = w > po / 2 ? -(double)(po - w) : (double)w;  // centred, exact
        const double wq = wc / (double)po;
        std::memcpy(&e[0], &wc, 8);
        std::memcpy(&e[1], &wq, 8);
      } else {
        e[0] = hmul(w, (uint64_t)(((u128)1 << 64) % po), po);  // Montgomery form
      }
    }
  }
  uint64_t* dcst = nullptr;
  int rc;
  if ((rc = dev_alloc(c, &dcst, std::max<size_t>(cst.size(), 1)))) return rc;
  HE_HIP(hipMemcpy(dcst, cst.data(), cst.size() * 8, hipMemcpyHostToDevice));
  t.cst = dcst;
  return HE_OK;
}

// Finishing constant of an inverse transform whose output feeds a basis
// conversion: N^{-1} (Qin/q_i)^{-1} mod q_i for input modulus m of a
// conversion with input moduli `ins`, as [integer, Shoup companion, double,
// double / q] in row m of a [L+K][4] table.
static void conv_fin_fill(const Ctx* c, const std::vector<int>& ins, int m, uint64_t* row) {
  const uint64_t q = c->mod[m];
  uint64_t prod = 1 % q;
  for (int m2 : ins)
    if (m2 != m) prod = hmul(prod, c->mod[m2] % q, q);
  const uint64_t w = hmul(hinv(prod, q), c->hmod[m].ninv, q);
  row[0] = w;
  row[1] = shoup_of(w, q);
  const double dw = (double)w, dwq = (double)w / (double)q;
  std::memcpy(&row[2], &dw, 8);
  std::memcpy(&row[3], &dwq, 8);
}

static int upload_set(Ctx* c, ConvSet& set, const std::vector<ConvDesc>& v) {
  set.count = (int)v.size();
  set.max_out = 0;
  set.max_parts = 0;
  set.max_in = 0;
  set.nout.clear();
  set.nint.clear();
  for (auto& d : v) {
    set.max_out = std::max(set.max_out, d.nout);
    set.max_parts = std::max(set.max_parts, d.nparts);
    set.max_in = std::max(set.max_in, d.nin);
    set.nout.push_back(d.nout);
    set.nint.push_back(d.nint);
  }
  int rc = dev_alloc(c, &set.d, v.size());
  if (rc) return rc;
  HE_HIP(hipMemcpy(set.d, v.data(), v.size() * sizeof(ConvDesc), hipMemcpyHostToDevice));
  return HE_OK;
}

static int ctx_init(Ctx* c, const he_params* p) {
  c->log_n = p->log_n;
  c->n = 1 << p->log_n;
  c->L = p->n_q;
  c->K = p->n_p;
  c->alpha = p->alpha;
  const uint64_t two_n = 2 * (uint64_t)c->n;
  // ---- primes
  std::vector<uint64_t> taken;
  std::map<int, uint64_t> next_k;
  auto take = [&](int b, uint64_t* out) -> int {
    if (b < 20 || b > 61) return set_error(HE_EINVAL, "prime bit size must be in [20, 61]");
    uint64_t k = next_k.count(b) ? next_k[b] : (((uint64_t)1 << b) - 2) / two_n;
    for (;; k--) {
      uint64_t q = k * two_n + 1;
      if (k == 0 || q <= ((uint64_t)1 << (b - 1))) return set_error(HE_EINVAL, "ran out of primes");
      if (q >= ((uint64_t)1 << b)) continue;
      bool used = false;
      for (uint64_t t : taken) used |= (t == q);
      if (used || !miller_rabin(q)) continue;
      taken.push_back(q);
      next_k[b] = k - 1;
      *out = q;
      return HE_OK;
    }
  };
  c->mod.assign(c->L + c->K, 0);
  for (int i = 0; i < c->L; i++) {
    if (p->q[i]) { c->mod[i] = p->q[i]; taken.push_back(p->q[i]); }
  }
  for (int k = 0; k < c->K; k++) {
    if (p->p[k]) { c->mod[c->L + k] = p->p[k]; taken.push_back(p->p[k]); }
  }
  for (int i = 0; i < c->L; i++)
    if (!c->mod[i]) { int rc = take(p->q_bits[i], &c->mod[i]); if (rc) return rc; }
  for (int k = 0; k < c->K; k++)
    if (!c->mod[c->L + k]) { int rc = take(p->p_bits[k], &c->mod[c->L + k]); if (rc) return rc; }
  for (uint64_t q : c->mod) {
    if (q >= ((uint64_t)1 << 61) || q % two_n != 1 || !miller_rabin(q))
      return set_error(HE_EINVAL, "every modulus must be a prime < 2^61 with q = 1 mod 2N");
  }
  // ---- per-modulus constants and twiddles
  const int M = c->L + c->K;
  const size_t N = c->n;
  c->psi.resize(M);
  c->hmod.resize(M);
  std::vector<uint64_t> tw(M * N), twp(M * N), itw(M * N), itwp(M * N), pw(N), ipw(N);
  std::vector<double> dtw(M * N), dtwq(M * N), ditw(M * N), ditwq(M * N);
  for (int m = 0; m < M; m++) {
    uint64_t q = c->mod[m];
    uint64_t psi = min_psi(q, N), ipsi = hinv(psi, q);
    c->psi[m] = psi;
    pw[0] = ipw[0] = 1;
    for (size_t k = 1; k < N; k++) { pw[k] = hmul(pw[k - 1], psi, q); ipw[k] = hmul(ipw[k - 1], ipsi, q); }
    for (size_t k = 0; k < N; k++) {
      int b = brv((int)k, c->log_n);
      tw[m * N + k] = pw[b];
      twp[m * N + k] = shoup_of(pw[b], q);
      itw[m * N + k] = ipw[b];
      itwp[m * N + k] = shoup_of(ipw[b], q);
      dtw[m * N + k] = (double)pw[b];
      dtwq[m * N + k] = (double)pw[b] / (double)q;
      ditw[m * N + k] = (double)ipw[b];
      ditwq[m * N + k] = (double)ipw[b] / (double)q;
    }
    ModInfo& mi = c->hmod[m];
    mi.q = q;
    uint64_t inv = 1;
    for (int it = 0; it < 7; it++) inv *= 2 - q * inv;  // Newton: q^{-1} mod 2^64
    mi.qinv = inv;
    uint64_t r64 = (uint64_t)(((u128)1 << 64) % q);
    mi.r2 = hmul(r64, r64, q);
    int kb = 64 - __builtin_clzll(q);
    mi.k = kb;
    mi.mu = (uint64_t)(((u128)1 << (2 * kb)) / q);
    mi.ninv = hinv(N % q, q);
    mi.ninv_p = shoup_of(mi.ninv, q);
    mi.pad = 0;
    mi.dninv = (double)mi.ninv;
    mi.dninvq = (double)mi.ninv / (double)q;
    mi.dqinv = 1.0 / (double)q;
    const uint64_t rinv = hinv(r64, q);  // 2^-64 mod q
    mi.drinv = (double)rinv;
    mi.drinvq = (double)rinv / (double)q;
    mi.dpad = 0.0;
  }
  int rc;
  if ((rc = dev_alloc(c, &c->d_mod, M))) return rc;
  if ((rc = dev_alloc(c, &c->d_tw, M * N))) return rc;
  if ((rc = dev_alloc(c, &c->d_twp, M * N))) return rc;
  if ((rc = dev_alloc(c, &c->d_itw, M * N))) return rc;
  if ((rc = dev_alloc(c, &c->d_itwp, M * N))) return rc;
  if ((rc = dev_alloc(c, &c->d_dtw, M * N))) return rc;
  if ((rc = dev_alloc(c, &c->d_dtwq, M * N))) return rc;
  if ((rc = dev_alloc(c, &c->d_ditw, M * N))) return rc;
  if ((rc = dev_alloc(c, &c->d_ditwq, M * N))) return rc;
  HE_HIP(hipMemcpy(c->d_mod, c->hmod.data(), M * sizeof(ModInfo), hipMemcpyHostToDevice));
  HE_HIP(hipMemcpy(c->d_tw, tw.data(), M * N * 8, hipMemcpyHostToDevice));
  HE_HIP(hipMemcpy(c->d_twp, twp.data(), M * N * 8, hipMemcpyHostToDevice));
  HE_HIP(hipMemcpy(c->d_itw, itw.data(), M * N * 8, hipMemcpyHostToDevice));
  HE_HIP(hipMemcpy(c->d_itwp, itwp.data(), M * N * 8, hipMemcpyHostToDevice));
  HE_HIP(hipMemcpy(c->d_dtw, dtw.data(), M * N * 8, hipMemcpyHostToDevice));
  HE_HIP(hipMemcpy(c->d_dtwq, dtwq.data(), M * N * 8, hipMemcpyHostToDevice));
  HE_HIP(hipMemcpy(c->d_ditw, ditw.data(), M * N * 8, hipMemcpyHostToDevice));
  HE_HIP(hipMemcpy(c->d_ditwq, ditwq.data(), M * N * 8, hipMemcpyHostToDevice));
  // ---- basis conversion tables for every level
  c->modup.assign(c->L + 1, {});
  c->moddown.assign(c->L + 1, {});
  c->rsconv.assign(c->L + 1, {});
  c->modup_ntt.assign(c->L + 1, LimbMap{});
  c->d_rescale.assign(c->L + 1, nullptr);
  c->d_pinv.assign(c->L + 1, nullptr);
  c->d_fin.assign(c->L + 1, nullptr);
  for (int l = 1; l <= c->L; l++) {
    int dn = c->dnum(l);
    const int E = l + c->K;
    std::vector<ConvDesc> ups(dn);
    LimbMap& nm = c->modup_ntt[l];
    nm.n = 0;
    // finishing constants of the inverse transforms feeding this level's
    // conversions: digit j's limbs for ModUp, the special primes for ModDown
    std::vector<uint64_t> fin((size_t)(c->L + c->K) * 4, 0);
    for (int j = 0; j < dn; j++) {
      std::vector<int> ip, im, op, om;
      int lo = j * c->alpha, hi = std::min((j + 1) * c->alpha, l);
      for (int i = lo; i < hi; i++) { ip.push_back(i); im.push_back(i); }
      for (int i = 0; i < l; i++)
        if (i < lo || i >= hi) { op.push_back(i); om.push_back(i); }
      for (int k = 0; k < c->K; k++) { op.push_back(l + k); om.push_back(c->L + k); }
      if ((rc = build_conv(c, ups[j], ip, im, op, om))) return rc;
      for (int m : im) conv_fin_fill(c, im, m, &fin[(size_t)m * 4]);
      for (size_t p = 0; p < op.size(); p++) {
        if (nm.n >= MAXJ) return set_error(HE_EINVAL, "too many extended limbs for one launch");
        nm.pos[nm.n] = (uint16_t)(j * E + op[p]);
        nm.mod[nm.n] = (uint8_t)om[p];
        nm.n++;
      }
    }
    if ((rc = upload_set(c, c->modup[l], ups))) return rc;
    std::vector<int> ip, im, op, om;
    for (int k = 0; k < c->K; k++) { ip.push_back(l + k); im.push_back(c->L + k); }
    for (int i = 0; i < l; i++) { op.push_back(i); om.push_back(i); }
    std::vector<ConvDesc> dn1(1);
    if ((rc = build_conv(c, dn1[0], ip, im, op, om))) return rc;
    if ((rc = upload_set(c, c->moddown[l], dn1))) return rc;
    for (int m : im) conv_fin_fill(c, im, m, &fin[(size_t)m * 4]);
    if ((rc = dev_alloc(c, &c->d_fin[l], fin.size()))) return rc;
    HE_HIP(hipMemcpy(c->d_fin[l], fin.data(), fin.size() * 8, hipMemcpyHostToDevice));
    // P^{-1} mod q_i
    std::vector<uint64_t> pv(2 * l);
    for (int i = 0; i < l; i++) {
      uint64_t qi = c->mod[i], P = 1;
      for (int k = 0; k < c->K; k++) P = hmul(P, c->mod[c->L + k] % qi, qi);
      pv[i] = hinv(P, qi);
      pv[l + i] = shoup_of(pv[i], qi);
    }
    // then, for the FP64 path of the fused ModDown epilogue, P^{-1} and P^{-1}/q as doubles
    pv.resize(4 * l);
    for (int i = 0; i < l; i++) {
      const double w = (double)pv[i], wq = (double)pv[i] / (double)c->mod[i];
      std::memcpy(&pv[2 * l + i], &w, 8);
      std::memcpy(&pv[3 * l + i], &wq, 8);
    }
    if ((rc = dev_alloc(c, &c->d_pinv[l], 4 * l))) return rc;
    HE_HIP(hipMemcpy(c->d_pinv[l], pv.data(), 4 * l * 8, hipMemcpyHostToDevice));
    if (l >= 2) {
      // rescale = ModDown by the single prime q_{l-1}: its conversion (one
      // input, constant 1) and q_{l-1}^{-1} in the epilogue's layout
      const int t = l - 1;
      std::vector<uint64_t> rv(4 * t);
      uint64_t qt = c->mod[t];
      for (int i = 0; i < t; i++) {
        rv[i] = hinv(qt % c->mod[i], c->mod[i]);
        rv[t + i] = shoup_of(rv[i], c->mod[i]);
        const double w = (double)rv[i], wq = (double)rv[i] / (double)c->mod[i];
        std::memcpy(&rv[2 * t + i], &w, 8);
        std::memcpy(&rv[3 * t + i], &wq, 8);
      }
      if ((rc = dev_alloc(c, &c->d_rescale[l], 4 * t))) return rc;
      HE_HIP(hipMemcpy(c->d_rescale[l], rv.data(), 4 * t * 8, hipMemcpyHostToDevice));
      std::vector<int> rin{0}, rim{t}, rop, rom;
      for (int i = 0; i < t; i++) { rop.push_back(i); rom.push_back(i); }
      std::vector<ConvDesc> rs1(1);
      if ((rc = build_conv(c, rs1[0], rin, rim, rop, rom))) return rc;
      if ((rc = upload_set(c, c->rsconv[l], rs1))) return rc;
    }
  }
  // ---- workspace: one top-level key switch + tensor + rescale scratch
  const size_t L = c->L, K = c->K, D = c->dnum(c->L);
  c->ws_words = ws_words(c);
  if ((rc = dev_alloc(c, &c->ws, c->ws_words))) return rc;
  c->key_words = D * 2 * (L + K) * N;
  if ((rc = ntt_autotune(c))) return rc;
  return conv_autotune(c);
}

Lane* lane_for(Ctx* c, hipStream_t s) {
  std::lock_guard<std::mutex> lk(c->lanes_mu);
  auto it = c->lanes.find(s);
  if (it != c->lanes.end()) return it->second;
  Lane* ln = new Lane();
  if (s == nullptr) {
    ln->ws = c->ws;
  } else {
    void* v = nullptr;
    if (hipMalloc(&v, c->ws_words * 8) != hipSuccess) {
      delete ln;
      set_error(HE_ENOMEM, "lane workspace allocation failed");
      return nullptr;
    }
    ln->ws = (uint64_t*)v;
  }
  c->lanes[s] = ln;
  return ln;
}

uint64_t* lane_ct_get(Ctx* c, Lane* ln) {
  if (!ln->ct_pool.empty()) {
    uint64_t* p = ln->ct_pool.back();
    ln->ct_pool.pop_back();
    return p;
  }
  void* v = nullptr;
  if (hipMalloc(&v, (size_t)2 * c->L * c->n * 8) != hipSuccess) {
    set_error(HE_ENOMEM, "ciphertext buffer allocation failed");
    return nullptr;
  }
  ln->ct_all.push_back((uint64_t*)v);
  return (uint64_t*)v;
}

static void lane_free(Ctx* c, hipStream_t s, Lane* ln) {
  for (uint64_t* p : ln->ct_all) hipFree(p);
  if (ln->set_ws) hipFree(ln->set_ws);
  if (ln->set_tab) hipFree(ln->set_tab);
  if (s != nullptr && ln->ws) hipFree(ln->ws);
  delete ln;
}

int aux_streams_for(Ctx* c, hipStream_t s, int n, hipStream_t* out) {
  std::lock_guard<std::mutex> lk(c->lanes_mu);
  std::vector<hipStream_t>& v = c->aux_streams[s];
  while ((int)v.size() < n) {
    hipStream_t a = nullptr;
    if (hipStreamCreateWithFlags(&a, hipStreamNonBlocking) != hipSuccess)
      return set_error(HE_EHIP, "helper stream creation failed");
    v.push_back(a);
  }
  for (int i = 0; i < n; i++) out[i] = v[i];
  return HE_OK;
}

bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return s && hipStreamIsCapturing(s, &st) == hipSuccess && st == hipStreamCaptureStatusActive;
}

int stream_fork(hipStream_t s, const hipStream_t* hs, int n) {
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return set_error(HE_EHIP, "event creation failed");
  hipError_t err = hipEventRecord(e, s);
  for (int i = 0; i < n && err == hipSuccess; i++) err = hipStreamWaitEvent(hs[i], e, 0);
  hipEventDestroy(e);
  return err == hipSuccess ? HE_OK : hip_error(err, "stream fork");
}

int stream_join(hipStream_t s, const hipStream_t* hs, int n) {
  int rc = HE_OK;
  for (int i = 0; i < n; i++) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      hipStreamSynchronize(hs[i]);  // cannot order on the device: wait on the host
      rc = set_error(HE_EHIP, "event creation failed");
      continue;
    }
    hipError_t err = hipEventRecord(e, hs[i]);
    if (err == hipSuccess) err = hipStreamWaitEvent(s, e, 0);
    if (err != hipSuccess) {
      hipStreamSynchronize(hs[i]);
      rc = hip_error(err, "stream join");
    }
    hipEventDestroy(e);
  }
  return rc;
}

// destroy the helper streams of caller stream s and their lanes (lanes_mu held)
static void aux_free(Ctx* c, hipStream_t s) {
  auto it = c->aux_streams.find(s);
  if (it == c->aux_streams.end()) return;
  for (hipStream_t a : it->second) {
    hipStreamSynchronize(a);
    auto ln = c->lanes.find(a);
    if (ln != c->lanes.end()) {
      lane_free(c, ln->first, ln->second);
      c->lanes.erase(ln);
    }
    hipStreamDestroy(a);
  }
  c->aux_streams.erase(it);
}

}  // namespace he

using namespace he;

extern "C" {

const char* he_last_error(void) { return g_err.c_str(); }

int he_lane_reserve(he_ctx* h, he_stream stream, int n_ct_buffers) {
  if (!h || n_ct_buffers < 0) return set_error(HE_EINVAL, "bad argument");
  Ctx* c = &h->c;
  Lane* ln = lane_for(c, (hipStream_t)stream);
  if (!ln) return HE_ENOMEM;
  std::vector<uint64_t*> got;
  for (int i = 0; i < n_ct_buffers; i++) {
    uint64_t* p = lane_ct_get(c, ln);
    if (!p) {
      for (uint64_t* q : got) ln->ct_pool.push_back(q);
      return HE_ENOMEM;
    }
    got.push_back(p);
  }
  for (uint64_t* q : got) ln->ct_pool.push_back(q);
  return HE_OK;
}

int he_lane_release(he_ctx* h, he_stream stream) {
  if (!h) return set_error(HE_EINVAL, "null context");
  Ctx* c = &h->c;
  HE_HIP(hipStreamSynchronize((hipStream_t)stream));
  std::lock_guard<std::mutex> lk(c->lanes_mu);
  aux_free(c, (hipStream_t)stream);
  auto it = c->lanes.find((hipStream_t)stream);
  if (it == c->lanes.end()) return HE_OK;
  lane_free(c, it->first, it->second);
  c->lanes.erase(it);
  return HE_OK;
}

size_t he_lane_bytes(const he_ctx* h, int n_ct_buffers) {
  if (!h) return 0;
  return h->c.ws_words * 8 + (size_t)n_ct_buffers * 2 * h->c.L * h->c.n * 8;
}

int he_ctx_create(const he_params* p, int device, he_ctx** out) {
  if (!p || !out) return set_error(HE_EINVAL, "null argument");
  *out = nullptr;
  if (p->log_n < 12 || p->log_n > 16 || p->log_n % 2)
    return set_error(HE_EINVAL, "log_n must be 12, 14 or 16");
  if (p->n_q < 1 || p->n_q > HE_MAX_Q || p->n_p < 1 || p->n_p > HE_MAX_P || p->n_q + p->n_p > MAXL)
    return set_error(HE_EINVAL, "bad number of primes");
  if (p->alpha < 1 || p->alpha > p->n_q || p->alpha > MAX_BCONV_IN || p->n_p > MAX_BCONV_IN)
    return set_error(HE_EINVAL, "alpha must be in [1, min(L, 10)] and K <= 10");
  if ((p->n_q + p->alpha - 1) / p->alpha > 8) return set_error(HE_EINVAL, "at most 8 key-switching digits");
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return hip_error(e, "hipSetDevice");
  he_ctx* h = new he_ctx();
  h->c.device = device;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
    h->c.lds_per_block = (size_t)lds;
  int rc = ctx_init(&h->c, p);
  if (rc) {
    he_ctx_destroy(h);
    return rc;
  }
  *out = h;
  return HE_OK;
}

int he_ctx_destroy(he_ctx* h) {
  if (!h) return HE_OK;
  hipSetDevice(h->c.device);
  hipDeviceSynchronize();
  keys_free_all(&h->c);
  {
    std::lock_guard<std::mutex> lk(h->c.lanes_mu);
    std::vector<hipStream_t> callers;
    for (auto& kv : h->c.aux_streams) callers.push_back(kv.first);
    for (hipStream_t st : callers) aux_free(&h->c, st);
  }
  for (auto& kv : h->c.lanes) lane_free(&h->c, kv.first, kv.second);
  h->c.lanes.clear();
  for (void* p : h->c.allocs) hipFree(p);
  delete h;
  return HE_OK;
}

int he_ctx_moduli(const he_ctx* h, uint64_t* out, int cap) {
  if (!h || !out) return set_error(HE_EINVAL, "null argument");
  int M = h->c.L + h->c.K;
  if (cap < M) return set_error(HE_EINVAL, "output too small");
  for (int i = 0; i < M; i++) out[i] = h->c.mod[i];
  return M;
}

int he_ctx_ntt_tuning(const he_ctx* h, int32_t* variant, float* us) {
  if (!h) return set_error(HE_EINVAL, "null context");
  for (int i = 0; i < 4; i++) {
    if (variant) variant[i] = h->c.ntt_var[i];
    for (int v = 0; v < NTT_VARIANTS; v++)
      if (us) us[v * 4 + i] = h->c.ntt_tune_us[v][i];
  }
  return HE_OK;
}

int he_ctx_conv_tuning(const he_ctx* h, int32_t* target, float* us) {
  if (!h) return set_error(HE_EINVAL, "null context");
  for (int k = 0; k < 2; k++) {
    if (target) target[k] = h->c.conv_target[k];
    for (int t = 0; t < 4; t++)
      if (us) us[k * 4 + t] = h->c.conv_tune_us[k][t];
  }
  return HE_OK;
}

int he_ctx_ntt_select(he_ctx* h, const int32_t* variant) {
  if (!h || !variant) return set_error(HE_EINVAL, "null argument");
  for (int i = 0; i < 4; i++)
    if (variant[i] < 0 || variant[i] >= NTT_VARIANTS) return set_error(HE_EINVAL, "bad NTT variant");
  for (int i = 0; i < 4; i++) h->c.ntt_var[i] = variant[i];
  return HE_OK;
}

int he_ntt_variant(int v, int32_t* tile, int32_t* per_thread) {
  if (v < 0 || v >= NTT_VARIANTS || !tile || !per_thread) return set_error(HE_EINVAL, "bad NTT variant");
  int t, e;
  ntt_variant_shape(v, &t, &e);
  *tile = t;
  *per_thread = e;
  return HE_OK;
}

int he_ctx_info(const he_ctx* h, int32_t* log_n, int32_t* n_q, int32_t* n_p, int32_t* alpha) {
  if (!h) return set_error(HE_EINVAL, "null argument");
  if (log_n) *log_n = h->c.log_n;
  if (n_q) *n_q = h->c.L;
  if (n_p) *n_p = h->c.K;
  if (alpha) *alpha = h->c.alpha;
  return HE_OK;
}

}  // extern "C"
