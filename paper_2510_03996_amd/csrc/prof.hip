// Per-kernel timing report (HIP events recorded around each launch).
#include <cstdio>
#include <cstring>
#include <map>
#include <string>

#include "internal.h"

using namespace he;

extern "C" {

int he_profile_begin(he_ctx* h) {
  if (!h) return set_error(HE_EINVAL, "null context");
  for (auto& r : h->c.prof) { hipEventDestroy(r.a); hipEventDestroy(r.b); }
  h->c.prof.clear();
  h->c.prof_on = true;
  return HE_OK;
}

int he_profile_end(he_ctx* h, char* out, size_t cap) {
  if (!h || !out || cap == 0) return set_error(HE_EINVAL, "null argument");
  Ctx* c = &h->c;
  c->prof_on = false;
  struct Agg { long n = 0; double ms = 0, bytes = 0, modmul = 0, ideal_ms = 0; };
  std::map<std::string, Agg> agg;
  for (auto& r : c->prof) {
    HE_HIP(hipEventSynchronize(r.b));
    float ms = 0;
    HE_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    Agg& a = agg[r.name];
    a.n++;
    a.ms += ms;
    a.bytes += r.bytes;
    a.modmul += r.modmul;
    a.ideal_ms += r.ideal_s * 1e3;
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  c->prof.clear();
  std::string js = "{";
  bool first = true;
  for (auto& kv : agg) {
    char buf[512];
    snprintf(buf, sizeof buf,
             "%s\"%s\": {\"launches\": %ld, \"ms\": %.6f, \"bytes\": %.0f, \"modmul\": %.0f, \"ideal_ms\": %.6f}",
             first ? "" : ", ", kv.first.c_str(), kv.second.n, kv.second.ms, kv.second.bytes, kv.second.modmul,
             kv.second.ideal_ms);
    js += buf;
    first = false;
  }
  js += "}";
  if (js.size() + 1 > cap) return set_error(HE_EINVAL, "report buffer too small");
  std::memcpy(out, js.c_str(), js.size() + 1);
  return (int)js.size();
}

}  // extern "C"
