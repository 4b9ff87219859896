// Evaluation-key store: resident keys, and the paper's dynamic key
// management (on-demand loading and removal) with device memory as a cache
// of keys whose pinned host copy the library holds.
//
// Ordering: a load is a host-to-device copy plus the Montgomery conversion on
// the stream of the operation that needs the key, followed by a `ready`
// event; another stream that uses the key before that event has completed
// waits for it.  Every kernel that reads a host-backed key is followed by a
// `used` event of its stream (one per stream that read the key), and an
// evicted key's buffer is handed to the next load only after all of them
// have completed, so no in-flight kernel on any stream ever reads a buffer
// that is being overwritten.  Replacing a key that has a device copy waits
// for the whole device.
#include <cstring>

#include "internal.h"

namespace he {

static size_t key_size(const Ctx* c) { return c->key_words * 8; }

static size_t resident_bytes(const Ctx* c) {
  size_t n = 0;
  for (auto& kv : c->keys) n += kv.second.dev ? key_size(c) : 0;
  return n;
}

static void destroy_events(KeyEntry& e) {
  for (auto& u : e.uses) hipEventDestroy(u.second);
  e.uses.clear();
  if (e.ready) hipEventDestroy(e.ready);
  e.ready = nullptr;
}

static void wait_and_free(Ctx* c, KeyEntry& e) {
  for (auto& u : e.uses) hipEventSynchronize(u.second);
  if (e.ready) hipEventSynchronize(e.ready);
  c->key_free.push_back(e.dev);
  e.dev = nullptr;
}

// A device buffer for a key about to be loaded: evict least recently used
// host-backed keys (not held by a batch, not `keep`) while the budget would be
// exceeded, then reuse a freed buffer or allocate one.
static uint64_t* key_buffer(Ctx* c, int32_t keep) {
  if (c->key_limit) {
    while (resident_bytes(c) + key_size(c) > c->key_limit) {
      KeyEntry* victim = nullptr;
      for (auto& kv : c->keys) {
        KeyEntry& e = kv.second;
        if (kv.first == keep || !e.dev || !e.host || e.locks > 0) continue;
        if (!victim || e.tick < victim->tick) victim = &e;
      }
      if (!victim) break;  // nothing evictable: the budget is exceeded
      wait_and_free(c, *victim);
      c->key_evictions++;
    }
  }
  if (!c->key_free.empty()) {
    uint64_t* d = c->key_free.back();
    c->key_free.pop_back();
    return d;
  }
  void* d = nullptr;
  if (hipMalloc(&d, key_size(c)) != hipSuccess) {
    set_error(HE_ENOMEM, "key allocation failed");
    return nullptr;
  }
  return (uint64_t*)d;
}

// copy src (host or device, plain form) into e.dev and convert to Montgomery form, on s
static int key_fill(Ctx* c, KeyEntry& e, const uint64_t* src, bool src_on_device, hipStream_t s) {
  HE_HIP(hipMemcpyAsync(e.dev, src, key_size(c), src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
  const int M = c->L + c->K;
  const int limbs = c->dnum(c->L) * 2 * M;
  k_to_mont<<<dim3(c->n / 256, limbs), 256, 0, s>>>(e.dev, M, c->log_n, c->d_mod);
  HE_HIP(hipGetLastError());
  if (!e.ready) HE_HIP(hipEventCreateWithFlags(&e.ready, hipEventDisableTiming));
  HE_HIP(hipEventRecord(e.ready, s));
  e.ready_stream = s;
  return HE_OK;
}

bool key_known(const Ctx* c, int32_t id) {
  auto it = c->keys.find(norm_key_id(c, id));
  return it != c->keys.end() && (it->second.dev || it->second.host);
}

const uint64_t* key_acquire(Ctx* c, int32_t id0, hipStream_t s) {
  const int32_t id = norm_key_id(c, id0);
  auto it = c->keys.find(id);
  if (it == c->keys.end() || (!it->second.dev && !it->second.host)) {
    set_error(HE_ENOKEY, "key " + std::to_string(id0) + " not available");
    return nullptr;
  }
  KeyEntry& e = it->second;
  if (e.host && stream_capturing(s)) {
    // loads, evictions and their host waits cannot be recorded into a graph
    set_error(HE_EUNSUPPORTED, "key " + std::to_string(id0) + " has a host copy: only resident keys can be captured");
    return nullptr;
  }
  e.tick = ++c->key_tick;
  if (!e.dev) {
    e.dev = key_buffer(c, id);
    if (!e.dev) return nullptr;
    if (key_fill(c, e, e.host, false, s)) return nullptr;
    c->key_loads++;
    return e.dev;
  }
  if (e.ready && e.ready_stream != s && hipEventQuery(e.ready) == hipErrorNotReady)
    if (hipStreamWaitEvent(s, e.ready, 0) != hipSuccess) {
      set_error(HE_EHIP, "stream wait on a key load failed");
      return nullptr;
    }
  return e.dev;
}

void key_note_use(Ctx* c, int32_t id, hipStream_t s) {
  auto it = c->keys.find(norm_key_id(c, id));
  if (it == c->keys.end() || !it->second.host) return;  // resident-only keys are never evicted
  KeyEntry& e = it->second;
  for (auto& u : e.uses)
    if (u.first == s) {
      hipEventRecord(u.second, s);
      return;
    }
  hipEvent_t ev = nullptr;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return;
  hipEventRecord(ev, s);
  e.uses.emplace_back(s, ev);
}

bool key_resident_only(const Ctx* c, int32_t id) {
  auto it = c->keys.find(norm_key_id(c, id));
  return it != c->keys.end() && it->second.dev && !it->second.host;
}

int key_lock(Ctx* c, int32_t id, int delta) {
  auto it = c->keys.find(norm_key_id(c, id));
  if (it == c->keys.end()) return HE_ENOKEY;
  it->second.locks += delta;
  return HE_OK;
}

void keys_free_all(Ctx* c) {
  for (auto& kv : c->keys) {
    KeyEntry& e = kv.second;
    if (e.dev) hipFree(e.dev);
    if (e.host) hipHostFree(e.host);
    destroy_events(e);
  }
  c->keys.clear();
  for (uint64_t* p : c->key_free) hipFree(p);
  c->key_free.clear();
}

}  // namespace he

using namespace he;

extern "C" {

int he_key_upload(he_ctx* h, int32_t key_id, const uint64_t* src, size_t bytes, int src_on_device, he_stream st) {
  if (!h || !src) return set_error(HE_EINVAL, "null argument");
  Ctx* c = &h->c;
  if (bytes != key_size(c)) return set_error(HE_EINVAL, "key size must be dnum*2*(L+K)*N*8 bytes");
  hipStream_t s = (hipStream_t)st;
  const int32_t id = norm_key_id(c, key_id);
  KeyEntry& e = c->keys[id];
  if (e.locks > 0) return set_error(HE_EINVAL, "key is held by a batch");
  e.tick = ++c->key_tick;
  if (!e.dev) {
    e.dev = key_buffer(c, id);
    if (!e.dev) {
      if (!e.host) c->keys.erase(id);
      return HE_ENOMEM;
    }
  } else {
    // the old contents may still be read by work enqueued on any stream
    HE_HIP(hipDeviceSynchronize());
  }
  int rc = key_fill(c, e, src, src_on_device != 0, s);
  if (rc) return rc;
  if (!src_on_device) HE_HIP(hipStreamSynchronize(s));  // host buffer may be freed after return
  if (e.host) {  // a host copy must match the device copy
    hipHostFree(e.host);
    e.host = nullptr;
  }
  return HE_OK;
}

int he_key_host_register(he_ctx* h, int32_t key_id, const uint64_t* src, size_t bytes) {
  if (!h || !src) return set_error(HE_EINVAL, "null argument");
  Ctx* c = &h->c;
  if (bytes != key_size(c)) return set_error(HE_EINVAL, "key size must be dnum*2*(L+K)*N*8 bytes");
  const int32_t id = norm_key_id(c, key_id);
  KeyEntry& e = c->keys[id];
  if (e.locks > 0) return set_error(HE_EINVAL, "key is held by a batch");
  if (!e.host) {
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes) != hipSuccess) {
      if (!e.dev) c->keys.erase(id);
      return set_error(HE_ENOMEM, "pinned host allocation failed");
    }
    e.host = (uint64_t*)p;
  }
  std::memcpy(e.host, src, bytes);
  if (e.dev) {  // a stale device copy is dropped; the next use loads the new key
    wait_and_free(c, e);
  }
  return HE_OK;
}

int he_key_cache_limit(he_ctx* h, size_t device_bytes) {
  if (!h) return set_error(HE_EINVAL, "null context");
  Ctx* c = &h->c;
  if (device_bytes && device_bytes < key_size(c)) return set_error(HE_EINVAL, "budget below one key");
  c->key_limit = device_bytes;
  return HE_OK;
}

int he_key_prefetch(he_ctx* h, const int32_t* ids, int n, he_stream st) {
  if (!h || (n > 0 && !ids) || n < 0) return set_error(HE_EINVAL, "bad arguments");
  Ctx* c = &h->c;
  for (int i = 0; i < n; i++)
    if (!key_known(c, ids[i])) return set_error(HE_ENOKEY, "key " + std::to_string(ids[i]) + " not available");
  for (int i = 0; i < n; i++)
    if (!key_acquire(c, ids[i], (hipStream_t)st)) return HE_ENOMEM;
  return HE_OK;
}

int he_key_cache_stats(const he_ctx* h, size_t* resident, int64_t* loads, int64_t* evictions) {
  if (!h) return set_error(HE_EINVAL, "null context");
  const Ctx* c = &h->c;
  if (resident) *resident = resident_bytes(c);
  if (loads) *loads = c->key_loads;
  if (evictions) *evictions = c->key_evictions;
  return HE_OK;
}

int he_key_evict(he_ctx* h, int32_t key_id) {
  if (!h) return set_error(HE_EINVAL, "null context");
  Ctx* c = &h->c;
  auto it = c->keys.find(norm_key_id(c, key_id));
  if (it == c->keys.end()) return set_error(HE_ENOKEY, "key not resident");
  KeyEntry& e = it->second;
  if (e.locks > 0) return set_error(HE_EINVAL, "key is held by a batch");
  HE_HIP(hipDeviceSynchronize());
  if (e.dev) hipFree(e.dev);
  if (e.host) hipHostFree(e.host);
  destroy_events(e);
  c->keys.erase(it);
  return HE_OK;
}

int he_key_count(const he_ctx* h) {
  if (!h) return 0;
  int n = 0;
  for (auto& kv : h->c.keys) n += kv.second.dev != nullptr;
  return n;
}

size_t he_key_bytes(const he_ctx* h) { return h ? key_size(&h->c) : 0; }

}  // extern "C"
