// NTT / iNTT kernels and launchers (see ntt_core.h for the decomposition).
#include "internal.h"
#include "ntt_core.h"

namespace he {

// grid: x = tile within limb, y = limb index in `map`, z = batch
template <int LOGN, int PASS, bool INV>
__global__ __launch_bounds__(256) void ntt_pass_kernel(const uint64_t* src, size_t src_bs, uint64_t* data,
                                                       size_t batch_stride, LimbMap map,
                                                       const uint64_t* __restrict__ tw_all,
                                                       const uint64_t* __restrict__ twp_all,
                                                       const double* __restrict__ dtw_all,
                                                       const double* __restrict__ dtwq_all,
                                                       const ModInfo* __restrict__ mods) {
  using P = NttPass<LOGN, PASS, INV>;
  __shared__ uint64_t lds[P::LDS_WORDS];
  const int wg = blockIdx.x;
  const int limb = blockIdx.y;
  const int tid = threadIdx.x;
  const int m = map.mod[limb];
  const uint64_t* ain = src + blockIdx.z * src_bs + (size_t)map.pos[limb] * P::N;
  uint64_t* a = data + blockIdx.z * batch_stride + (size_t)map.pos[limb] * P::N;
  const uint64_t* tw = tw_all + (size_t)m * P::N;
  const uint64_t* twp = twp_all + (size_t)m * P::N;
  const ModInfo mi = mods[m];
  const uint64_t q = mi.q;
  if (mi.k <= 50) {
    // FP64 path (exact doubles, full-rate FMA products); the branch is uniform per workgroup
    double* dl = reinterpret_cast<double*>(lds);
    const double* dtw = dtw_all + (size_t)m * P::N;
    const double* dtwq = dtwq_all + (size_t)m * P::N;
    const double dq = (double)q;
    for (int e = tid; e < P::TILE; e += P::THREADS) {
      int g, k;
      P::tile_elem(e, g, k);
      dl[P::lidx(g, k)] = (double)ain[P::gidx(wg, g, k)];
    }
    __syncthreads();
    if (!INV) {
      P::template round_f64<P::R1>(dl, tid, wg, 0, dtw, dtwq, dq);
      if (P::R2 > 0) {
        __syncthreads();
        P::template round_f64<(P::R2 > 0 ? P::R2 : 1)>(dl, tid, wg, P::R1, dtw, dtwq, dq);
      }
    } else {
      if (P::R2 > 0) {
        P::template round_f64<(P::R2 > 0 ? P::R2 : 1)>(dl, tid, wg, P::R1, dtw, dtwq, dq);
        __syncthreads();
      }
      P::template round_f64<P::R1>(dl, tid, wg, 0, dtw, dtwq, dq);
    }
    __syncthreads();
    for (int e = tid; e < P::TILE; e += P::THREADS) {
      int g, k;
      P::tile_elem(e, g, k);
      a[P::gidx(wg, g, k)] = P::finish_f64(dl[P::lidx(g, k)], mi.dninv, mi.dninvq, dq);
    }
    return;
  }
  for (int e = tid; e < P::TILE; e += P::THREADS) {
    int g, k;
    P::tile_elem(e, g, k);
    lds[P::lidx(g, k)] = ain[P::gidx(wg, g, k)];
  }
  __syncthreads();
  if (!INV) {
    P::template round<P::R1>(lds, tid, wg, 0, tw, twp, q);
    if (P::R2 > 0) {
      __syncthreads();
      P::template round<(P::R2 > 0 ? P::R2 : 1)>(lds, tid, wg, P::R1, tw, twp, q);
    }
  } else {
    if (P::R2 > 0) {
      P::template round<(P::R2 > 0 ? P::R2 : 1)>(lds, tid, wg, P::R1, tw, twp, q);
      __syncthreads();
    }
    P::template round<P::R1>(lds, tid, wg, 0, tw, twp, q);
  }
  __syncthreads();
  for (int e = tid; e < P::TILE; e += P::THREADS) {
    int g, k;
    P::tile_elem(e, g, k);
    a[P::gidx(wg, g, k)] = P::finish(lds[P::lidx(g, k)], mi.ninv, mi.ninv_p, q);
  }
}

template <int LOGN>
static int ntt_launch_n(Ctx* c, const uint64_t* src, size_t src_bs, uint64_t* data, size_t batch_stride,
                        int nbatch, const LimbMap& map, bool inverse, hipStream_t s) {
  using P1 = NttPass<LOGN, 1, false>;
  using P2 = NttPass<LOGN, 2, false>;
  dim3 g1(P1::WG_PER_LIMB, map.n, nbatch), g2(P2::WG_PER_LIMB, map.n, nbatch);
  const double limbs = (double)map.n * nbatch, N = (double)P1::N;
  const double bytes = 16.0 * N * limbs;  // one read + one write of every residue per pass
  const double mm1 = N / 2 * P1::LM * limbs, mm2 = N / 2 * P2::LM * limbs;
  if (!inverse) {
    {
      ProfScope ps(c, "ntt_fwd_pass1", s, bytes, mm1);
      ntt_pass_kernel<LOGN, 1, false><<<g1, 256, 0, s>>>(src, src_bs, data, batch_stride, map, c->d_tw, c->d_twp, c->d_dtw,
                                                             c->d_dtwq, c->d_mod);
    }
    ProfScope ps(c, "ntt_fwd_pass2", s, bytes, mm2);
    ntt_pass_kernel<LOGN, 2, false><<<g2, 256, 0, s>>>(data, batch_stride, data, batch_stride, map, c->d_tw, c->d_twp,
                                                             c->d_dtw, c->d_dtwq, c->d_mod);
  } else {
    {
      ProfScope ps(c, "ntt_inv_pass2", s, bytes, mm2);
      ntt_pass_kernel<LOGN, 2, true><<<g2, 256, 0, s>>>(src, src_bs, data, batch_stride, map, c->d_itw, c->d_itwp,
                                                         c->d_ditw, c->d_ditwq, c->d_mod);
    }
    ProfScope ps(c, "ntt_inv_pass1", s, bytes, mm1 + N * limbs);
    ntt_pass_kernel<LOGN, 1, true><<<g1, 256, 0, s>>>(data, batch_stride, data, batch_stride, map, c->d_itw, c->d_itwp,
                                                            c->d_ditw, c->d_ditwq, c->d_mod);
  }
  HE_HIP(hipGetLastError());
  return HE_OK;
}

int ntt_launch_strided(Ctx* c, const uint64_t* src, size_t src_bs, uint64_t* data, size_t batch_stride, int nbatch,
                       const LimbMap& map, bool inverse, hipStream_t s) {
  if (map.n <= 0 || nbatch <= 0) return HE_OK;
  if (nbatch > 65535) return set_error(HE_EINVAL, "NTT batch too large for one launch");
  switch (c->log_n) {
    case 12: return ntt_launch_n<12>(c, src, src_bs, data, batch_stride, nbatch, map, inverse, s);
    case 14: return ntt_launch_n<14>(c, src, src_bs, data, batch_stride, nbatch, map, inverse, s);
    case 16: return ntt_launch_n<16>(c, src, src_bs, data, batch_stride, nbatch, map, inverse, s);
  }
  return set_error(HE_EINVAL, "unsupported ring degree");
}

int ntt_launch_from(Ctx* c, const uint64_t* src, uint64_t* data, size_t batch_stride, int nbatch, const LimbMap& map,
                    bool inverse, hipStream_t s) {
  return ntt_launch_strided(c, src, batch_stride, data, batch_stride, nbatch, map, inverse, s);
}

int ntt_launch(Ctx* c, uint64_t* data, size_t batch_stride, int nbatch, const LimbMap& map, bool inverse,
               hipStream_t s) {
  return ntt_launch_from(c, data, data, batch_stride, nbatch, map, inverse, s);
}

}  // namespace he

using namespace he;

extern "C" int he_ntt(he_ctx* h, uint64_t* poly, int n_limbs, int first_limb, int inverse, he_stream stream) {
  if (!h || !poly) return set_error(HE_EINVAL, "null argument");
  Ctx* c = &h->c;
  if (n_limbs < 0 || first_limb < 0 || first_limb + n_limbs > c->L + c->K)
    return set_error(HE_EINVAL, "limb range outside the moduli");
  return ntt_launch(c, poly, 0, 1, range_map(0, n_limbs, first_limb), inverse != 0, (hipStream_t)stream);
}
