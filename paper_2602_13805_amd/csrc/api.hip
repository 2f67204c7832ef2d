// C ABI of the PDF hot path: handle setup, the per-iteration launch sequence,
// the start value, images and the reconstruction loop.
#include <hip/hip_runtime.h>

#include <array>
#include <chrono>
#include <map>
#include <memory>
#include <mutex>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include "cco_loss_kernels.h"
#include "conv_big.h"
#include "conv_kernels.h"
#include "fcnn_kernels.h"
#include "handle.h"
#include "init_kernels.h"
#include "mf_kernels.h"
#include "pixel_kernels.h"
#include "tables.h"

using namespace pdfk;

static thread_local std::string g_last_error = "no error";

// Device memory for entry points that allocate nothing (pdf_init_alpha_csi_noalloc).
// Each device holds its own copy of this array from the first use of the
// library until the process ends.  In host code its name is not a device
// address: kernels receive the address that hipGetSymbolAddress returns for
// the current device (scratch_address), never the name itself.
static __device__ __align__(256) unsigned char scratch[PDF_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Address of `scratch` on the current device (looked up once per device).
static hipError_t scratch_address(int dev, void** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

#define HIP_TRY(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      return fail(h, PDF_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    }                                                                              \
  } while (0)

void pdf_set_global_error(const std::string& msg) { g_last_error = msg; }

static int fail(pdf_handle* h, int code, const std::string& msg) {
  if (h)
    h->err_msg = msg;
  else
    g_last_error = msg;
  return code;
}

static int check_launch(pdf_handle* h, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(h, PDF_EHIP, std::string("launch ") + what + ": " + hipGetErrorString(e));
  return PDF_OK;
}

extern "C" int pdf_default_params(pdf_params* p) {
  if (!p) return PDF_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->version = PDF_PARAMS_VERSION;
  p->precision = PDF_FP32;
  p->beta = 6.0;
  p->lam_bound = 1e-3;
  p->lam_tv = 1e-5;
  p->lam_bridge = 1e-5;
  p->tau_b = 0.5;
  p->eps_tv = 1e-12;
  p->eps_abs = 1e-12;
  p->cco_tau = 3.0;
  p->cco_eta_max = 0.1;
  p->cco_delta = 0.5;
  p->gf_radius = 1;
  p->gf_eps = 1e-2;
  p->lr = 1e-2;
  p->adam_b1 = 0.9;
  p->adam_b2 = 0.999;
  p->adam_eps = 1e-8;
  p->r_stopgrad = 0;
  return PDF_OK;
}

static bool supported_m(int prec, int M) {
  return M == 8 || M == 16 || M == 32 || M == 48 || M == 64 || M == 96 || M == 128 || M == 256;
}

// Grids whose convolution runs in passes through global memory (conv_big.h):
// the padded half tile exceeds one CU's LDS.
static bool big_grid(int prec, int M) { return prec == PDF_FP32 ? M >= 128 : M >= 96; }

// ------------------------------------------------------------------ launchers

template <typename K>
static void set_lds(K kernel, size_t bytes) {
  if (bytes > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              int(bytes));
}

// The band-limited forward and adjoint on the compact tile: FP32 at 64 x 64 with K <= 32;
// with K <= 16 the adjoint keeps the row transform of g_J, and the forward beta U, in the
// tile's spare columns.
static bool fwd_compact(const pdf_handle* h) {
  return h->prec == PDF_FP32 && h->M == 64 && !h->big && h->K <= CompactCfg<float, 64>::KC;
}
static bool adj_gj_spare(const pdf_handle* h) { return fwd_compact(h) && 2 * h->K <= CompactCfg<float, 64>::KC; }
static int compact_mode(const pdf_handle* h) { return fwd_compact(h) ? (adj_gj_spare(h) ? 2 : 1) : 0; }

template <typename T, int M, bool FA, bool PP>
static void launch_fwd_t(pdf_handle* h, const FwdArgs<T>& a, int nblk) {
  using C = ConvCfg<T, M>;
  auto k = k_fwd_conv<T, M, FA, PP>;
  set_lds(k, C::fwd_lds(PP, FA));
  hipLaunchKernelGGL(k, dim3(nblk), dim3(C::NT), C::fwd_lds(PP, FA), h->stream, a);
}

template <typename T, int M>
static int launch_fwd_m(pdf_handle* h, const FwdArgs<T>& a, bool from_alpha, int nblk) {
  using C = ConvCfg<T, M>;
  if constexpr (sizeof(T) == 4 && M == 64) {
    if (from_alpha && fwd_compact(h)) {  // every plan choice: one kernel from coefficients
      using CC = CompactCfg<T, M>;
      if (adj_gj_spare(h)) {
        set_lds(k_fwd_conv_c<T, M, true>, CC::LDS);
        hipLaunchKernelGGL((k_fwd_conv_c<T, M, true>), dim3(nblk), dim3(CC::NT), CC::LDS, h->stream, a);
      } else {
        set_lds(k_fwd_conv_c<T, M, false>, CC::LDS);
        hipLaunchKernelGGL((k_fwd_conv_c<T, M, false>), dim3(nblk), dim3(CC::NT), CC::LDS, h->stream, a);
      }
      return check_launch(h, "k_fwd_conv_c");
    }
  }
  if constexpr (C::fwd_lds(false, true) <= 160 * 1024) {
    // FP64 handles keep the default plan (no tuning there)
    const bool pp = sizeof(T) == 4 && h->tune_fpp != 0;
    if constexpr (sizeof(T) == 4 && C::fwd_lds(true, true) <= 160 * 1024) {
      if (pp) {
        if (from_alpha)
          launch_fwd_t<T, M, true, true>(h, a, nblk);
        else
          launch_fwd_t<T, M, false, true>(h, a, nblk);
        return check_launch(h, "k_fwd_conv");
      }
    }
    if (from_alpha)
      launch_fwd_t<T, M, true, false>(h, a, nblk);
    else
      launch_fwd_t<T, M, false, false>(h, a, nblk);
    return check_launch(h, "k_fwd_conv");
  } else {
    return fail(h, PDF_EUNSUPPORTED, "grid too large for the LDS-resident convolution");
  }
}

// ---- grids beyond one CU's LDS: the convolution in three passes through S

template <typename T, int M>
static int launch_fwd_big_m(pdf_handle* h, const FwdArgs<T>& a, bool from_alpha) {
  using C = BigCfg<T, M>;
  const int bp = h->B * h->Ni;
  cx<T>* S = (cx<T>*)h->S;
  if (from_alpha) {
    set_lds(k_big_rows_fwd<T, M, true>, C::ROW_LDS);
    hipLaunchKernelGGL((k_big_rows_fwd<T, M, true>), dim3(bp * C::RBLK), dim3(C::NT), C::ROW_LDS, h->stream, a, S);
  } else {
    set_lds(k_big_rows_fwd<T, M, false>, C::ROW_LDS);
    hipLaunchKernelGGL((k_big_rows_fwd<T, M, false>), dim3(bp * C::RBLK), dim3(C::NT), C::ROW_LDS, h->stream, a, S);
  }
  set_lds(k_big_cols<T, M>, C::COL_LDS);
  hipLaunchKernelGGL((k_big_cols<T, M>), dim3(bp * C::CBLK), dim3(C::NTC), C::COL_LDS, h->stream, a.ghat, a.tw, S, 0);
  if (from_alpha) {
    set_lds(k_big_rows_inv<T, M, true>, C::ROW_LDS);
    hipLaunchKernelGGL((k_big_rows_inv<T, M, true>), dim3(bp * C::RBLK), dim3(C::NT), C::ROW_LDS, h->stream, a,
                       (const cx<T>*)S);
  } else {
    set_lds(k_big_rows_inv<T, M, false>, C::ROW_LDS);
    hipLaunchKernelGGL((k_big_rows_inv<T, M, false>), dim3(bp * C::RBLK), dim3(C::NT), C::ROW_LDS, h->stream, a,
                       (const cx<T>*)S);
  }
  return check_launch(h, "big-grid forward convolution");
}

template <typename T>
static int launch_fwd_big(pdf_handle* h, const FwdArgs<T>& a, bool from_alpha) {
  switch (h->M) {
    case 128: return launch_fwd_big_m<T, 128>(h, a, from_alpha);
    case 256: return launch_fwd_big_m<T, 256>(h, a, from_alpha);
    case 96:
      if constexpr (sizeof(T) == 8) return launch_fwd_big_m<T, 96>(h, a, from_alpha);
      break;
  }
  return fail(h, PDF_EUNSUPPORTED, "unsupported M for the big-grid convolution");
}

// The analysis half of the adjoint for the K kept modes of the rows in S plus
// g_J (src = null), or of the pixel arrays src: row transforms, then the
// column DFT with the gradient output and Adam of a, results times scale.
template <typename T, int M>
static int launch_adj_tail_big_m(pdf_handle* h, const AdjArgs<T>& a, int npairs, const cx<T>* src, T scale) {
  using C = BigCfg<T, M>;
  cx<T>* S = (cx<T>*)h->S;
  if (!src) {
    set_lds(k_big_adj_rows_inv<T, M, true>, C::ROW_LDS);
    hipLaunchKernelGGL((k_big_adj_rows_inv<T, M, true>), dim3(npairs * C::RBLK), dim3(C::NT), C::ROW_LDS, h->stream,
                       a.tw, S, (const cx<T>*)h->GJ, a.K);
  } else {
    set_lds(k_big_adj_rows_inv<T, M, false>, C::ROW_LDS);
    hipLaunchKernelGGL((k_big_adj_rows_inv<T, M, false>), dim3(npairs * C::RBLK), dim3(C::NT), C::ROW_LDS,
                       h->stream, a.tw, S, src, a.K);
  }
  // the kept rows split over up to 8 workgroups per pair
  hipLaunchKernelGGL((k_big_adj_final<T, M>), dim3(npairs, a.K < 8 ? a.K : 8), dim3(256), sizeof(cx<T>) * C::P,
                     h->stream, a, (const cx<T>*)S, scale);
  return check_launch(h, "big-grid analysis");
}

template <typename T, int M>
static int launch_adj_big_m(pdf_handle* h, const AdjArgs<T>& a) {
  using C = BigCfg<T, M>;
  const int bp = h->B * h->Ni;
  cx<T>* S = (cx<T>*)h->S;
  set_lds(k_big_adj_rows<T, M>, C::ROW_LDS);
  hipLaunchKernelGGL((k_big_adj_rows<T, M>), dim3(bp * C::RBLK), dim3(C::NT), C::ROW_LDS, h->stream, a, S,
                     (cx<T>*)h->GJ);
  set_lds(k_big_cols<T, M>, C::COL_LDS);
  hipLaunchKernelGGL((k_big_cols<T, M>), dim3(bp * C::CBLK), dim3(C::NTC), C::COL_LDS, h->stream, a.ghat, a.tw, S, 1);
  int rc = check_launch(h, "big-grid adjoint convolution");
  if (rc) return rc;
  return launch_adj_tail_big_m<T, M>(h, a, bp, nullptr, T(1));
}

template <typename T>
static int launch_adj_big(pdf_handle* h, const AdjArgs<T>& a) {
  switch (h->M) {
    case 128: return launch_adj_big_m<T, 128>(h, a);
    case 256: return launch_adj_big_m<T, 256>(h, a);
    case 96:
      if constexpr (sizeof(T) == 8) return launch_adj_big_m<T, 96>(h, a);
      break;
  }
  return fail(h, PDF_EUNSUPPORTED, "unsupported M for the big-grid adjoint");
}

template <typename T>
static int launch_fwd(pdf_handle* h, const FwdArgs<T>& a, bool from_alpha) {
  if (from_alpha && !a.J)  // the coefficient path keeps J in its output between phases
    return fail(h, PDF_EINVAL, "internal: coefficient synthesis without a J buffer");
  if (h->big) return launch_fwd_big<T>(h, a, from_alpha);
  const int nblk = h->B * h->Ni;
  switch (h->M) {
    case 8: return launch_fwd_m<T, 8>(h, a, from_alpha, nblk);
    case 16: return launch_fwd_m<T, 16>(h, a, from_alpha, nblk);
    case 32: return launch_fwd_m<T, 32>(h, a, from_alpha, nblk);
    case 48: return launch_fwd_m<T, 48>(h, a, from_alpha, nblk);
    case 64: return launch_fwd_m<T, 64>(h, a, from_alpha, nblk);
    case 96: return launch_fwd_m<T, 96>(h, a, from_alpha, nblk);
  }
  return fail(h, PDF_EUNSUPPORTED, "unsupported M");
}

template <typename T, int M, bool PP>
static void launch_adj_t(pdf_handle* h, const AdjArgs<T>& a, int nblk) {
  using C = ConvCfg<T, M>;
  auto k = k_adj_conv<T, M, PP>;
  set_lds(k, C::adj_lds(PP));
  hipLaunchKernelGGL(k, dim3(nblk), dim3(C::NT), C::adj_lds(PP), h->stream, a);
}

template <typename T, int M>
static int launch_adj_m(pdf_handle* h, const AdjArgs<T>& a, int nblk) {
  using C = ConvCfg<T, M>;
  if constexpr (sizeof(T) == 4 && M == 64) {
    if (fwd_compact(h)) {  // every plan choice: the band-limited adjoint on the compact tile
      using CC = CompactCfg<T, M>;
      if (adj_gj_spare(h)) {
        set_lds(k_adj_conv_c<T, M, true>, CC::LDS_ADJ);
        hipLaunchKernelGGL((k_adj_conv_c<T, M, true>), dim3(nblk), dim3(CC::NT), CC::LDS_ADJ, h->stream, a);
      } else {
        set_lds(k_adj_conv_c<T, M, false>, CC::LDS_ADJ);
        hipLaunchKernelGGL((k_adj_conv_c<T, M, false>), dim3(nblk), dim3(CC::NT), CC::LDS_ADJ, h->stream, a);
      }
      return check_launch(h, "k_adj_conv_c");
    }
  }
  if constexpr (C::adj_lds(false) <= 160 * 1024) {
    if constexpr (sizeof(T) == 4 && C::adj_lds(true) <= 160 * 1024) {
      if (h->tune_app != 0) {
        launch_adj_t<T, M, true>(h, a, nblk);
        return check_launch(h, "k_adj_conv");
      }
    }
    launch_adj_t<T, M, false>(h, a, nblk);
    return check_launch(h, "k_adj_conv");
  } else {
    return fail(h, PDF_EUNSUPPORTED, "grid too large for the LDS-resident convolution");
  }
}

template <typename T>
static int launch_adj(pdf_handle* h, const AdjArgs<T>& a) {
  if (h->big) return launch_adj_big<T>(h, a);
  const int nblk = h->B * h->Ni;
  switch (h->M) {
    case 8: return launch_adj_m<T, 8>(h, a, nblk);
    case 16: return launch_adj_m<T, 16>(h, a, nblk);
    case 32: return launch_adj_m<T, 32>(h, a, nblk);
    case 48: return launch_adj_m<T, 48>(h, a, nblk);
    case 64: return launch_adj_m<T, 64>(h, a, nblk);
    case 96: return launch_adj_m<T, 96>(h, a, nblk);
  }
  return fail(h, PDF_EUNSUPPORTED, "unsupported M");
}

template <int NRT, int NCT>
static void launch_reduce_mfma(pdf_handle* h, const ReduceArgs<float>& a) {
  const size_t lds = reduce_mfma_lds<NCT>();
  if (h->tune_pb == 8) {
    set_lds(k_pixel_reduce_mfma<NRT, NCT, 8>, lds);
    hipLaunchKernelGGL((k_pixel_reduce_mfma<NRT, NCT, 8>), dim3(h->ntiles, h->B), dim3(256), lds, h->stream, a);
  } else {
    set_lds(k_pixel_reduce_mfma<NRT, NCT, 4>, lds);
    hipLaunchKernelGGL((k_pixel_reduce_mfma<NRT, NCT, 4>), dim3(h->ntiles, h->B), dim3(256), lds, h->stream, a);
  }
}

template <typename T>
static ReduceArgs<T> reduce_args(pdf_handle* h, const cx<T>* J, const cx<T>* E, const cx<T>* Rfix) {
  ReduceArgs<T> a;
  a.J = J;
  a.E = E;
  a.gs = (const cx<T>*)h->gs;
  a.gsT = (const cx<T>*)h->gsT;
  a.gsA = h->gsA;
  a.Rfix = Rfix;
  a.R = (cx<T>*)h->R;
  a.den = (T*)h->den;
  a.chi = (cx<T>*)h->chi;
  a.lsp = h->lsp;
  a.Dpart = (cx<T>*)h->Dpart;
  a.wsum = h->mf_wsum;
  a.wgt = h->mf_w;
  a.Ni = h->Ni;
  a.Ns = h->Ns;
  a.N = h->N;
  a.ntiles = h->ntiles;
  a.beta = T(h->prm.beta);
  return a;
}

template <typename T>
static int launch_reduce(pdf_handle* h, const cx<T>* J, const cx<T>* E, const cx<T>* Rfix) {
  const ReduceArgs<T> a = reduce_args<T>(h, J, E, Rfix);
  if constexpr (sizeof(T) == 4) {
    const int nrt = (h->Ns + 15) / 16, nct = (h->Ni + 31) / 32;
    switch (nct * 8 + nrt) {
      case 9: launch_reduce_mfma<1, 1>(h, a); break;
      case 10: launch_reduce_mfma<2, 1>(h, a); break;
      case 11: launch_reduce_mfma<3, 1>(h, a); break;
      case 12: launch_reduce_mfma<4, 1>(h, a); break;
      case 17: launch_reduce_mfma<1, 2>(h, a); break;
      case 18: launch_reduce_mfma<2, 2>(h, a); break;
      case 19: launch_reduce_mfma<3, 2>(h, a); break;
      case 20: launch_reduce_mfma<4, 2>(h, a); break;
      default: return fail(h, PDF_EUNSUPPORTED, "incidence / receiver count out of range");
    }
    return check_launch(h, "k_pixel_reduce_mfma");
  } else {
    const size_t lds = sizeof(cx<T>) * size_t(h->Ni) * h->tile + 16 * sizeof(double);
    set_lds(k_pixel_reduce<T>, lds);
    hipLaunchKernelGGL(k_pixel_reduce<T>, dim3(h->ntiles, h->B), dim3(h->tile), lds, h->stream, a);
    return check_launch(h, "k_pixel_reduce");
  }
}

template <typename T>
static RegArgs<T> reg_args(pdf_handle* h, double* loss, int* tstep, const int* frozen) {
  RegArgs<T> a;
  a.nfreq = h->F;
  a.dn = h->dn;
  a.sdf = h->sdf;
  a.chi = (const cx<T>*)h->chi;
  a.R = (const cx<T>*)h->R;
  a.Dpart = (const cx<T>*)h->Dpart;
  a.lsp = h->lsp;
  a.esca = (const cx<T>*)h->esca;
  a.Ss = h->Ss;
  a.Sd = h->Sd;
  a.d = (cx<T>*)h->dres;
  a.gR = (cx<T>*)h->gR;
  a.loss = loss;
  a.tstep = tstep;
  a.frozen = frozen;
  a.adam_c = h->adam_c;
  a.lr = h->prm.lr;
  a.b1 = h->prm.adam_b1;
  a.b2 = h->prm.adam_b2;
  a.M = h->M;
  a.Ni = h->Ni;
  a.Ns = h->Ns;
  a.ntiles = h->ntiles;
  a.beta = h->prm.beta;
  a.lam_bound = h->prm.lam_bound;
  a.lam_tv = h->prm.lam_tv;
  a.lam_bridge = h->prm.lam_bridge;
  a.tau_b = h->prm.tau_b;
  a.eps_tv = h->prm.eps_tv;
  a.eps_abs = h->prm.eps_abs;
  a.r_stopgrad = h->prm.r_stopgrad;
  a.lse = nullptr;
  a.nlse = 0;
  a.graw = 0;
  return a;
}

// The loss on the CCO image: chi_c and R_c from chi, the regularisers on chi_c
// (their dL/dchi_c kept unconverted in gR), then the gradient back through the
// CCO to g_R (unless R is held fixed).
template <typename T>
static int launch_reg_cco(pdf_handle* h, RegArgs<T> a) {
  const int N = h->N, nblk = (N + 255) / 256;
  CcoLossArgs<T> c;
  c.chi = (const cx<T>*)h->chi;
  c.R = (const cx<T>*)h->R;
  c.den = (const T*)h->den;
  c.Ss = h->Ss;
  c.ws = (T*)h->ccl_ws;
  c.chic = (cx<T>*)h->chic;
  c.Rc = (cx<T>*)h->Rc;
  c.part = h->ccl_part;
  c.g = (cx<T>*)h->gR;
  c.loss = a.loss;
  c.M = h->M;
  c.r = h->prm.gf_radius;
  c.r_stopgrad = h->prm.r_stopgrad;
  c.beta = h->prm.beta;
  c.gf_eps = h->prm.gf_eps;
  c.tau = h->prm.cco_tau;
  c.eta_max = h->prm.cco_eta_max;
  c.delta = h->prm.cco_delta;
  const dim3 grid(nblk, h->B);
  hipLaunchKernelGGL(k_ccl_coef<T>, grid, dim3(256), 0, h->stream, c);
  hipLaunchKernelGGL(k_ccl_apply<T>, grid, dim3(256), 0, h->stream, c);
  int rc = check_launch(h, "k_ccl_coef/apply");
  if (rc) return rc;
  a.chi = c.chic;
  a.lse = h->ccl_part;
  a.nlse = nblk;
  a.graw = h->prm.r_stopgrad ? 0 : 1;
  const size_t lds = 2 * sizeof(cx<T>) * size_t(N) + 16 * sizeof(double);
  set_lds(k_image_reg<T>, lds);
  hipLaunchKernelGGL(k_image_reg<T>, dim3(h->B), dim3(N < 1024 ? N : 1024), lds, h->stream, a);
  if ((rc = check_launch(h, "k_image_reg"))) return rc;
  if (h->prm.r_stopgrad) return PDF_OK;  // g_R = 0, written by the regulariser pass
  hipLaunchKernelGGL(k_ccl_adj1<T>, grid, dim3(256), 0, h->stream, c);
  hipLaunchKernelGGL(k_ccl_adj2<T>, grid, dim3(256), 0, h->stream, c);
  hipLaunchKernelGGL(k_ccl_adj3<T>, grid, dim3(256), 0, h->stream, c);
  return check_launch(h, "k_ccl_adj");
}

template <typename T>
static int launch_reg(pdf_handle* h, double* loss, int* tstep, const int* frozen) {
  const RegArgs<T> a = reg_args<T>(h, loss, tstep, frozen);
  if (h->prm.cco_in_loss) return launch_reg_cco<T>(h, a);
  const int nt = h->N < 1024 ? h->N : 1024;
  if (h->big) {  // chi read from global memory, 256 pixels per workgroup
    const int nblk = (h->N + 255) / 256;
    hipLaunchKernelGGL(k_image_reg_part<T>, dim3(nblk, h->B), dim3(256), 0, h->stream, a, h->reg_part);
    hipLaunchKernelGGL(k_image_reg_fin<T>, dim3(h->B), dim3(256), 0, h->stream, a, (const double*)h->reg_part, nblk);
    return check_launch(h, "k_image_reg_part/fin");
  }
  if (h->N > reg_pix_max<T>() * nt) return fail(h, PDF_EUNSUPPORTED, "grid too large for the one-workgroup regulariser");
  const size_t lds = 2 * sizeof(cx<T>) * size_t(h->N) + 16 * sizeof(double);
  set_lds(k_image_reg<T>, lds);
  hipLaunchKernelGGL(k_image_reg<T>, dim3(h->B), dim3(nt), lds, h->stream, a);
  return check_launch(h, "k_image_reg");
}

template <int NRT, int CT>
static void launch_adj_gemm_ct(pdf_handle* h, const cx<float>* x, cx<float>* out) {
  const size_t lds = sizeof(cx<float>) * size_t(h->Ns) * 16 * NRT;
  constexpr int px = 4 * 32 * CT;  // pixels per workgroup
  dim3 grid((h->N + px - 1) / px, h->B);
  hipLaunchKernelGGL((k_adj_gemm_mfma<NRT, CT>), grid, dim3(256), lds, h->stream, (const cx<float>*)h->gs, x, out,
                     h->Ni, h->Ns, h->N);
}

template <int NRT>
static void launch_adj_gemm_mfma(pdf_handle* h, const cx<float>* x, cx<float>* out) {
  switch (h->tune_ct) {
    case 1: launch_adj_gemm_ct<NRT, 1>(h, x, out); break;
    case 4: launch_adj_gemm_ct<NRT, 4>(h, x, out); break;
    default: launch_adj_gemm_ct<NRT, 2>(h, x, out); break;
  }
}

template <typename T>
static int launch_adj_gemm(pdf_handle* h, const cx<T>* x, cx<T>* out) {
  if constexpr (sizeof(T) == 4) {
    if (h->N % 32 == 0) {
      switch ((h->Ni + 15) / 16) {
        case 1: launch_adj_gemm_mfma<1>(h, x, out); break;
        case 2: launch_adj_gemm_mfma<2>(h, x, out); break;
        case 3: launch_adj_gemm_mfma<3>(h, x, out); break;
        case 4: launch_adj_gemm_mfma<4>(h, x, out); break;
        default: return fail(h, PDF_EUNSUPPORTED, "incidence count out of range");
      }
      return check_launch(h, "k_adj_gemm_mfma");
    }
  }
  const size_t lds = sizeof(cx<T>) * size_t(h->Ni) * h->Ns;
  dim3 grid((h->N + 255) / 256, h->B);
  if (h->Ns <= 16)
    hipLaunchKernelGGL((k_adj_gemm<T, 16>), grid, dim3(256), lds, h->stream, (const cx<T>*)h->gs, x, out, h->Ni,
                       h->Ns, h->N);
  else if (h->Ns <= 32)
    hipLaunchKernelGGL((k_adj_gemm<T, 32>), grid, dim3(256), lds, h->stream, (const cx<T>*)h->gs, x, out, h->Ni,
                       h->Ns, h->N);
  else
    hipLaunchKernelGGL((k_adj_gemm<T, 64>), grid, dim3(256), lds, h->stream, (const cx<T>*)h->gs, x, out, h->Ni,
                       h->Ns, h->N);
  return check_launch(h, "k_adj_gemm");
}

// Records the next timing event on the handle's stream (no-op unless timing).
static int mark(pdf_handle* h) {
  // the pool holds whole steps, so a step is either recorded fully or not at all
  if (!h->timing || h->ev_used >= int(h->events.size())) return PDF_OK;
  HIP_TRY(hipEventRecord(h->events[h->ev_used], h->stream));
  h->ev_used++;
  return PDF_OK;
}

template <typename T>
static FwdArgs<T> fwd_args(pdf_handle* h, const void* alpha) {
  FwdArgs<T> f;
  f.in = (const cx<T>*)alpha;
  f.einc = (const cx<T>*)h->einc;
  f.ghat = (const cx<T>*)h->ghat;
  f.tw = (const cx<T>*)h->tw;
  f.J = (cx<T>*)h->J;
  f.E = (cx<T>*)h->E;
  f.Ni = h->Ni;
  f.K = h->K;
  f.beta = T(h->prm.beta);
  return f;
}

template <typename T>
static AdjArgs<T> adj_args(pdf_handle* h, void* grad, void* alpha_upd, void* m, void* v, const int* frozen) {
  AdjArgs<T> a;
  a.J = (const cx<T>*)h->J;
  a.E = (const cx<T>*)h->E;
  a.e_shared = 0;
  a.h = (const cx<T>*)h->h;
  a.R = (const cx<T>*)h->R;
  a.Rs = nullptr;
  a.den = (const T*)h->den;
  a.gR = (const cx<T>*)h->gR;
  a.Ss = h->Ss;
  a.Sd = h->Sd;
  a.hsign = 1.0;
  a.ghat = (const cx<T>*)h->ghat;
  a.tw = (const cx<T>*)h->tw;
  a.galpha = (cx<T>*)grad;
  a.alpha = (cx<T>*)alpha_upd;
  a.m = (T*)m;
  a.v = (T*)v;
  a.frozen = frozen;
  a.gr_w = T(1);
  a.adam_c = h->adam_c;
  a.b1 = h->prm.adam_b1;
  a.b2 = h->prm.adam_b2;
  a.eps = h->prm.adam_eps;
  a.Ni = h->Ni;
  a.K = h->K;
  a.beta = T(h->prm.beta);
  return a;
}

// Several frequencies (defined below, after the single-frequency runners they call).
template <typename T>
static int run_iteration_mf(pdf_handle* h, const void* alpha, void* grad, double* loss, void* alpha_upd, void* m,
                            void* v, int* tstep, const int* frozen);
template <typename T>
static int mf_forward(pdf_handle* h, const void* alpha);
template <typename T>
static int run_init_mf(pdf_handle* h, void* alpha_out);
template <typename T>
static int launch_reg(pdf_handle* h, double* loss, int* tstep, const int* frozen);

// One evaluation of loss and gradient; with Adam buffers, also the update.
template <typename T>
static int run_iteration(pdf_handle* h, const void* alpha, void* grad, double* loss, void* alpha_upd, void* m,
                         void* v, int* tstep, const int* frozen) {
  if (h->F > 1) return run_iteration_mf<T>(h, alpha, grad, loss, alpha_upd, m, v, tstep, frozen);
  int rc;
  const FwdArgs<T> f = fwd_args<T>(h, alpha);
  if ((rc = mark(h))) return rc;
  if ((rc = launch_fwd<T>(h, f, true))) return rc;
  if ((rc = mark(h))) return rc;
  if ((rc = launch_reduce<T>(h, (const cx<T>*)h->J, (const cx<T>*)h->E, nullptr))) return rc;
  if ((rc = mark(h))) return rc;
  if ((rc = launch_reg<T>(h, loss, tstep, frozen))) return rc;
  if ((rc = mark(h))) return rc;
  if ((rc = launch_adj_gemm<T>(h, (const cx<T>*)h->dres, (cx<T>*)h->h))) return rc;
  if ((rc = mark(h))) return rc;
  AdjArgs<T> a = adj_args<T>(h, grad, alpha_upd, m, v, frozen);
  if (h->prm.cco_in_loss) a.Rs = (const cx<T>*)h->Rc;  // the state residual's contrast
  if ((rc = launch_adj<T>(h, a))) return rc;
  return mark(h);
}

// ------------------------------------------------------------------ grouped launches

// FP32 handles of one shape class (grid M, receiver tiles ceil(Ns/16),
// incidence tiles ceil(Ni/32) and ceil(Ni/16), tile choice) advanced by one
// launch per kernel: each launch reads a table of the handles' argument sets
// and the first workgroup of each set.  The handles may differ in N_i, N_s,
// K and batch within the class.
struct Group {
  std::vector<pdf_handle*> hs;
  void* dmem = nullptr;
  const FwdArgs<float>* fwd = nullptr;
  const ReduceArgs<float>* red = nullptr;
  const RegArgs<float>* reg = nullptr;
  const AdjGemmArgs* ag = nullptr;
  const AdjArgs<float>* adj = nullptr;
  const int* st[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // [n + 1] workgroup starts per kernel
  int tot[5] = {0, 0, 0, 0, 0};
  int n = 0, M = 0, ntiles = 0, nbx = 0, nt_reg = 0, nrt = 0, nct = 0, nrta = 0, ct = 2, pb = 4, fpp = 0, app = 0;
  int compact = 0;  // compact_mode of every member (one class)
  size_t lds_reg = 0, lds_ag = 0;
  ~Group() {
    if (dmem) (void)hipFree(dmem);
  }
};

// Caller-owned step state of each member (pdf_step_multi); absent: the handles' own
// reconstruction state (pdf_reconstruct_multi).
struct StepBufs {
  std::vector<void*> m, v;
  std::vector<int*> t;
  std::vector<double*> loss;
};

static int group_build(Group* g, const std::vector<pdf_handle*>& hs, const std::vector<void*>& alphas,
                       const StepBufs* bufs = nullptr) {
  pdf_handle* h0 = hs[0];
  g->hs = hs;
  g->n = int(hs.size());
  g->M = h0->M;
  g->ntiles = h0->ntiles;
  g->nrt = (h0->Ns + 15) / 16;
  g->nct = (h0->Ni + 31) / 32;
  g->nrta = (h0->Ni + 15) / 16;
  g->ct = h0->tune_ct;
  g->compact = compact_mode(h0);
  for (pdf_handle* h : hs)
    if (compact_mode(h) != g->compact) return fail(h0, PDF_EINVAL, "internal: one class, one convolution tile");
  g->pb = h0->tune_pb;
  g->fpp = h0->tune_fpp;
  g->app = h0->tune_app;
  g->nbx = (h0->N + 128 * g->ct - 1) / (128 * g->ct);
  g->nt_reg = h0->N < 1024 ? h0->N : 1024;
  g->lds_reg = 2 * sizeof(cx<float>) * size_t(h0->N) + 16 * sizeof(double);
  int max_ns = 0;
  for (pdf_handle* h : hs) max_ns = std::max(max_ns, h->Ns);
  g->lds_ag = sizeof(cx<float>) * size_t(max_ns) * 16 * g->nrta;
  const int n = g->n;
  std::vector<FwdArgs<float>> fwd(n);
  std::vector<ReduceArgs<float>> red(n);
  std::vector<RegArgs<float>> reg(n);
  std::vector<AdjGemmArgs> ag(n);
  std::vector<AdjArgs<float>> adj(n);
  std::vector<int> st(5 * size_t(n + 1), 0);
  for (int i = 0; i < n; ++i) {
    pdf_handle* h = hs[i];
    fwd[i] = fwd_args<float>(h, alphas[i]);
    red[i] = reduce_args<float>(h, (const cx<float>*)h->J, (const cx<float>*)h->E, nullptr);
    reg[i] = bufs ? reg_args<float>(h, bufs->loss[i], bufs->t[i], nullptr) : reg_args<float>(h, h->loss, h->tstep, h->frozen);
    ag[i] = AdjGemmArgs{(const cx<float>*)h->gs, (const cx<float>*)h->dres, (cx<float>*)h->h, h->Ni, h->Ns, h->N};
    adj[i] = bufs ? adj_args<float>(h, nullptr, alphas[i], bufs->m[i], bufs->v[i], nullptr)
                  : adj_args<float>(h, nullptr, alphas[i], h->m, h->v, h->frozen);
    const int cnt[5] = {h->B * h->Ni, h->ntiles * h->B, h->B, g->nbx * h->B, h->B * h->Ni};
    for (int k = 0; k < 5; ++k) st[k * size_t(n + 1) + i + 1] = st[k * size_t(n + 1) + i] + cnt[k];
  }
  for (int k = 0; k < 5; ++k) g->tot[k] = st[k * size_t(n + 1) + n];
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t o1 = al(sizeof(FwdArgs<float>) * n), o2 = o1 + al(sizeof(ReduceArgs<float>) * n),
               o3 = o2 + al(sizeof(RegArgs<float>) * n), o4 = o3 + al(sizeof(AdjGemmArgs) * n),
               o5 = o4 + al(sizeof(AdjArgs<float>) * n), total = o5 + sizeof(int) * st.size();
  std::vector<unsigned char> hostbuf(total, 0);
  std::memcpy(hostbuf.data(), fwd.data(), sizeof(FwdArgs<float>) * n);
  std::memcpy(hostbuf.data() + o1, red.data(), sizeof(ReduceArgs<float>) * n);
  std::memcpy(hostbuf.data() + o2, reg.data(), sizeof(RegArgs<float>) * n);
  std::memcpy(hostbuf.data() + o3, ag.data(), sizeof(AdjGemmArgs) * n);
  std::memcpy(hostbuf.data() + o4, adj.data(), sizeof(AdjArgs<float>) * n);
  std::memcpy(hostbuf.data() + o5, st.data(), sizeof(int) * st.size());
  pdf_handle* h = h0;
  HIP_TRY(hipMalloc(&g->dmem, total));
  HIP_TRY(hipMemcpy(g->dmem, hostbuf.data(), total, hipMemcpyHostToDevice));
  unsigned char* d = static_cast<unsigned char*>(g->dmem);
  g->fwd = reinterpret_cast<const FwdArgs<float>*>(d);
  g->red = reinterpret_cast<const ReduceArgs<float>*>(d + o1);
  g->reg = reinterpret_cast<const RegArgs<float>*>(d + o2);
  g->ag = reinterpret_cast<const AdjGemmArgs*>(d + o3);
  g->adj = reinterpret_cast<const AdjArgs<float>*>(d + o4);
  for (int k = 0; k < 5; ++k) g->st[k] = reinterpret_cast<const int*>(d + o5) + k * size_t(n + 1);
  return PDF_OK;
}

template <int M, bool PP>
static void group_conv_t(const Group* g, hipStream_t st, bool adjoint) {
  using C = ConvCfg<float, M>;
  if (!adjoint) {
    auto k = k_fwd_conv_group<float, M, true, PP>;
    set_lds(k, C::fwd_lds(PP, true));
    hipLaunchKernelGGL(k, dim3(g->tot[0]), dim3(C::NT), C::fwd_lds(PP, true), st, g->fwd, g->st[0], g->n);
  } else {
    auto k = k_adj_conv_group<float, M, PP>;
    set_lds(k, C::adj_lds(PP));
    hipLaunchKernelGGL(k, dim3(g->tot[4]), dim3(C::NT), C::adj_lds(PP), st, g->adj, g->st[4], g->n);
  }
}

template <int M>
static void group_conv_m(const Group* g, hipStream_t st, bool adjoint) {
  using C = ConvCfg<float, M>;
  if constexpr (C::adj_lds(false) <= 160 * 1024) {
    if constexpr (C::adj_lds(true) <= 160 * 1024) {
      if ((adjoint ? g->app : g->fpp) != 0) {
        group_conv_t<M, true>(g, st, adjoint);
        return;
      }
    }
    group_conv_t<M, false>(g, st, adjoint);
  }
}

static void group_conv(const Group* g, hipStream_t st, bool adjoint) {
  if (g->compact) {
    using CC = CompactCfg<float, 64>;
    if (!adjoint && g->compact == 2) {
      set_lds(k_fwd_conv_c_group<float, 64, true>, CC::LDS);
      hipLaunchKernelGGL((k_fwd_conv_c_group<float, 64, true>), dim3(g->tot[0]), dim3(CC::NT), CC::LDS, st, g->fwd,
                         g->st[0], g->n);
    } else if (!adjoint) {
      set_lds(k_fwd_conv_c_group<float, 64, false>, CC::LDS);
      hipLaunchKernelGGL((k_fwd_conv_c_group<float, 64, false>), dim3(g->tot[0]), dim3(CC::NT), CC::LDS, st, g->fwd,
                         g->st[0], g->n);
    } else if (g->compact == 2) {
      set_lds(k_adj_conv_c_group<float, 64, true>, CC::LDS_ADJ);
      hipLaunchKernelGGL((k_adj_conv_c_group<float, 64, true>), dim3(g->tot[4]), dim3(CC::NT), CC::LDS_ADJ, st, g->adj,
                         g->st[4], g->n);
    } else {
      set_lds(k_adj_conv_c_group<float, 64, false>, CC::LDS_ADJ);
      hipLaunchKernelGGL((k_adj_conv_c_group<float, 64, false>), dim3(g->tot[4]), dim3(CC::NT), CC::LDS_ADJ, st, g->adj,
                         g->st[4], g->n);
    }
    return;
  }
  switch (g->M) {
    case 8: group_conv_m<8>(g, st, adjoint); break;
    case 16: group_conv_m<16>(g, st, adjoint); break;
    case 32: group_conv_m<32>(g, st, adjoint); break;
    case 48: group_conv_m<48>(g, st, adjoint); break;
    case 64: group_conv_m<64>(g, st, adjoint); break;
    case 96: group_conv_m<96>(g, st, adjoint); break;
  }
}

template <int NRT, int NCT>
static void group_reduce_t(const Group* g, hipStream_t st) {
  const size_t lds = reduce_mfma_lds<NCT>();
  if (g->pb == 8) {
    set_lds(k_pixel_reduce_mfma_group<NRT, NCT, 8>, lds);
    hipLaunchKernelGGL((k_pixel_reduce_mfma_group<NRT, NCT, 8>), dim3(g->tot[1]), dim3(256), lds, st, g->red,
                       g->st[1], g->n, g->ntiles);
  } else {
    set_lds(k_pixel_reduce_mfma_group<NRT, NCT, 4>, lds);
    hipLaunchKernelGGL((k_pixel_reduce_mfma_group<NRT, NCT, 4>), dim3(g->tot[1]), dim3(256), lds, st, g->red,
                       g->st[1], g->n, g->ntiles);
  }
}

static void group_reduce(const Group* g, hipStream_t st) {
  switch (g->nct * 8 + g->nrt) {
    case 9: group_reduce_t<1, 1>(g, st); break;
    case 10: group_reduce_t<2, 1>(g, st); break;
    case 11: group_reduce_t<3, 1>(g, st); break;
    case 12: group_reduce_t<4, 1>(g, st); break;
    case 17: group_reduce_t<1, 2>(g, st); break;
    case 18: group_reduce_t<2, 2>(g, st); break;
    case 19: group_reduce_t<3, 2>(g, st); break;
    case 20: group_reduce_t<4, 2>(g, st); break;
  }
}

template <int NRT, int CT>
static void group_adj_gemm_t(const Group* g, hipStream_t st) {
  hipLaunchKernelGGL((k_adj_gemm_mfma_group<NRT, CT>), dim3(g->tot[3]), dim3(256), g->lds_ag, st, g->ag, g->st[3],
                     g->n, g->nbx);
}

template <int NRT>
static void group_adj_gemm_n(const Group* g, hipStream_t st) {
  switch (g->ct) {
    case 1: group_adj_gemm_t<NRT, 1>(g, st); break;
    case 4: group_adj_gemm_t<NRT, 4>(g, st); break;
    default: group_adj_gemm_t<NRT, 2>(g, st); break;
  }
}

static void group_adj_gemm(const Group* g, hipStream_t st) {
  switch (g->nrta) {
    case 1: group_adj_gemm_n<1>(g, st); break;
    case 2: group_adj_gemm_n<2>(g, st); break;
    case 3: group_adj_gemm_n<3>(g, st); break;
    case 4: group_adj_gemm_n<4>(g, st); break;
  }
}

// k grouped iterations (loss, gradient, Adam) on the first handle's stream.
static int group_iterate(const Group* g, int k) {
  pdf_handle* h = g->hs[0];
  hipStream_t st = h->stream;
  set_lds(k_image_reg_group<float>, g->lds_reg);
  for (int s = 0; s < k; ++s) {
    group_conv(g, st, false);
    group_reduce(g, st);
    hipLaunchKernelGGL(k_image_reg_group<float>, dim3(g->tot[2]), dim3(g->nt_reg), g->lds_reg, st, g->reg,
                       g->st[2], g->n);
    group_adj_gemm(g, st);
    group_conv(g, st, true);
  }
  return check_launch(h, "grouped iteration");
}

// Loss only (no adjoint): forward kernels and the image / regulariser pass.
template <typename T>
static int run_loss(pdf_handle* h, const void* alpha, double* loss) {
  int rc;
  if (h->F > 1) {
    if ((rc = mf_forward<T>(h, alpha))) return rc;
    return launch_reg<T>(h, loss, nullptr, nullptr);
  }
  FwdArgs<T> f;
  f.in = (const cx<T>*)alpha;
  f.einc = (const cx<T>*)h->einc;
  f.ghat = (const cx<T>*)h->ghat;
  f.tw = (const cx<T>*)h->tw;
  f.J = (cx<T>*)h->J;
  f.E = (cx<T>*)h->E;
  f.Ni = h->Ni;
  f.K = h->K;
  f.beta = T(h->prm.beta);
  if ((rc = launch_fwd<T>(h, f, true))) return rc;
  if ((rc = launch_reduce<T>(h, (const cx<T>*)h->J, (const cx<T>*)h->E, nullptr))) return rc;
  return launch_reg<T>(h, loss, nullptr, nullptr);
}

template <typename T>
static int run_image(pdf_handle* h, const void* alpha, void* chi_out, void* cco_out, const void* eps_true,
                     double* err) {
  int rc;
  if (h->F > 1) {
    if ((rc = mf_forward<T>(h, alpha))) return rc;
  } else {
    FwdArgs<T> f;
    f.in = (const cx<T>*)alpha;
    f.einc = (const cx<T>*)h->einc;
    f.ghat = (const cx<T>*)h->ghat;
    f.tw = (const cx<T>*)h->tw;
    f.J = (cx<T>*)h->J;
    f.E = (cx<T>*)h->E;
    f.Ni = h->Ni;
    f.K = h->K;
    f.beta = T(h->prm.beta);
    if ((rc = launch_fwd<T>(h, f, true))) return rc;
    if ((rc = launch_reduce<T>(h, (const cx<T>*)h->J, (const cx<T>*)h->E, nullptr))) return rc;
  }
  if (chi_out)
    HIP_TRY(hipMemcpyAsync(chi_out, h->chi, sizeof(cx<T>) * size_t(h->B) * h->N, hipMemcpyDeviceToDevice,
                           h->stream));
  if (cco_out || err) {
    CcoArgs<T> c;
    c.chi = (const cx<T>*)h->chi;
    c.out = (cx<T>*)cco_out;
    c.eps_true = (const cx<T>*)eps_true;
    c.err = eps_true ? err : nullptr;
    c.M = h->M;
    c.r = h->prm.gf_radius;
    c.gf_eps = h->prm.gf_eps;
    c.tau = h->prm.cco_tau;
    c.eta_max = h->prm.cco_eta_max;
    c.delta = h->prm.cco_delta;
    if (h->big) {
      // coefficients, then the image and per-workgroup error sums, then the errors
      T* w = (T*)h->big_ws;
      const int nblk = (h->N + 255) / 256;
      double* part = reinterpret_cast<double*>(w + size_t(h->B) * 4 * h->N);
      hipLaunchKernelGGL(k_cco_big_coef<T>, dim3(nblk, h->B), dim3(256), 0, h->stream, (const cx<T>*)h->chi, w, h->M,
                         c.r, c.gf_eps);
      hipLaunchKernelGGL(k_cco_big_apply<T>, dim3(nblk, h->B), dim3(256), 0, h->stream, (const cx<T>*)h->chi,
                         (const T*)w, c, part);
      if (c.err) hipLaunchKernelGGL(k_cco_big_err, dim3(h->B), dim3(1), 0, h->stream, (const double*)part, nblk, c.err);
      return check_launch(h, "k_cco_big");
    }
    const int nt = h->N < 1024 ? h->N : 1024;
    if (h->N > kCcoPix * 1024) return fail(h, PDF_EUNSUPPORTED, "grid too large for the CCO kernel");
    const size_t lds = 4 * sizeof(T) * size_t(h->N) + 16 * sizeof(double);
    set_lds(k_cco<T>, lds);
    hipLaunchKernelGGL(k_cco<T>, dim3(h->B), dim3(nt), lds, h->stream, c);
    if ((rc = check_launch(h, "k_cco"))) return rc;
  }
  return PDF_OK;
}

// Start value (Sec. 3.1): BP image, R_0, single exact-line-search step on L^CSI.
template <typename T>
static int run_init(pdf_handle* h, void* alpha_out) {
  if (h->F > 1) return run_init_mf<T>(h, alpha_out);
  int rc;
  cx<T>* u = (cx<T>*)h->h;
  // u_p = G_S^H e_p
  if ((rc = launch_adj_gemm<T>(h, (const cx<T>*)h->esca, u))) return rc;
  // v_p = G_S u_p (split-K parts), gamma_p, J_BP = gamma_p u_p
  if ((rc = launch_reduce<T>(h, u, u, nullptr))) return rc;
  hipLaunchKernelGGL(k_bp_gamma<T>, dim3(h->B * h->Ni), dim3(256), 0, h->stream, (const cx<T>*)h->Dpart,
                     h->ntiles, (const cx<T>*)h->esca, u, h->Ni, h->Ns, h->N);
  if ((rc = check_launch(h, "k_bp_gamma"))) return rc;
  // E = E_inc + G_D J_BP
  FwdArgs<T> f;
  f.in = u;
  f.einc = (const cx<T>*)h->einc;
  f.ghat = (const cx<T>*)h->ghat;
  f.tw = (const cx<T>*)h->tw;
  f.J = nullptr;
  f.E = (cx<T>*)h->E;
  f.Ni = h->Ni;
  f.K = h->K;
  f.beta = T(0);
  if ((rc = launch_fwd<T>(h, f, false))) return rc;
  hipLaunchKernelGGL(k_bp_contrast<T>, dim3((h->N + 255) / 256, h->B), dim3(256), 0, h->stream, (const cx<T>*)u,
                     (const cx<T>*)h->E, (cx<T>*)h->R0, h->Ni, h->N, h->prm.beta);
  if ((rc = check_launch(h, "k_bp_contrast"))) return rc;
  // g = grad L^CSI(0): the adjoint with J = 0, E = E_inc, R = R_0 fixed, d = -e
  if ((rc = launch_adj_gemm<T>(h, (const cx<T>*)h->esca, u))) return rc;
  AdjArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  a.J = nullptr;
  a.E = (const cx<T>*)h->einc;
  a.e_shared = 1;
  a.h = u;
  a.R = (const cx<T>*)h->R0;
  a.den = nullptr;
  a.gR = nullptr;
  a.Ss = h->Ss;
  a.Sd = h->Sd;
  a.hsign = -1.0;
  a.ghat = (const cx<T>*)h->ghat;
  a.tw = (const cx<T>*)h->tw;
  a.galpha = (cx<T>*)h->g0;
  a.alpha = nullptr;
  a.gr_w = T(1);
  a.Ni = h->Ni;
  a.K = h->K;
  a.beta = T(h->prm.beta);
  if ((rc = launch_adj<T>(h, a))) return rc;
  const size_t kk = size_t(h->K) * h->K;
  hipLaunchKernelGGL(k_sumsq<T>, dim3(h->B), dim3(256), 0, h->stream, (const cx<T>*)h->g0, size_t(h->Ni) * kk,
                     h->gnorm);
  if ((rc = check_launch(h, "k_sumsq"))) return rc;
  // curvature along g: J_g = F_T^*(g), A_s g = R_0 (G_D J_g + beta J_g) - beta J_g, A_d g = G_S J_g
  f.in = (const cx<T>*)h->g0;
  f.einc = nullptr;
  f.J = (cx<T>*)h->J;
  f.E = (cx<T>*)h->E;
  f.beta = T(h->prm.beta);
  if ((rc = launch_fwd<T>(h, f, true))) return rc;
  if ((rc = launch_reduce<T>(h, (const cx<T>*)h->J, (const cx<T>*)h->E, (const cx<T>*)h->R0))) return rc;
  hipLaunchKernelGGL(k_line_search<T>, dim3(h->B), dim3(256), 0, h->stream, h->lsp, (const cx<T>*)h->Dpart,
                     h->ntiles, h->Ni, h->Ns, h->gnorm, h->Ss, h->Sd, (const cx<T>*)h->g0, (cx<T>*)alpha_out,
                     int(kk));
  return check_launch(h, "k_line_search");
}

// The full CSI start: n_iter conjugate-gradient steps on L^CSI from zero (the
// first is run_init's exact steepest-descent step).  Per further step: the
// gradient at alpha (forward with E_inc, the reduction with R_0 fixed, the
// data residual, G_S^H, the adjoint without an R-gradient), the conjugate
// direction, its curvature (forward without E_inc, reduction with R_0) and
// the exact step.
static size_t csi_align(size_t x) { return (x + 255) & ~size_t(255); }

// Bytes of the conjugate-gradient workspace: the direction [B][Ni][K][K] and two
// doubles per instance.  Every value in it is written before it is read within
// one call, so it needs no clearing.
static size_t csi_workspace_bytes(const pdf_handle* h) {
  const size_t csz = h->prec == PDF_FP32 ? sizeof(cx<float>) : sizeof(cx<double>);
  return csi_align(csz * h->B * size_t(h->Ni) * h->K * h->K) + 2 * csi_align(sizeof(double) * h->B);
}

// ws: device workspace of csi_workspace_bytes(h) bytes (unused when n_iter == 1).
template <typename T>
static int run_csi(pdf_handle* h, int n_iter, void* alpha_out, void* ws) {
  int rc;
  if ((rc = run_init<T>(h, alpha_out))) return rc;
  if (n_iter <= 1) return PDF_OK;
  const size_t len = size_t(h->Ni) * h->K * h->K;
  auto al = csi_align;
  unsigned char* w = static_cast<unsigned char*>(ws);
  cx<T>* p = reinterpret_cast<cx<T>*>(w);
  double* gprev = reinterpret_cast<double*>(w + al(sizeof(cx<T>) * h->B * len));
  double* dot = gprev + al(sizeof(double) * h->B) / sizeof(double);
  cx<T>* alpha = (cx<T>*)alpha_out;
  const cx<T>* R0 = (const cx<T>*)h->R0;
  const int NO = h->Ni * h->Ns;
  hipLaunchKernelGGL(k_csi_dir<T>, dim3(h->B), dim3(256), 0, h->stream, (const cx<T>*)h->g0, p, h->gnorm, gprev, dot,
                     len, 1);
  if ((rc = check_launch(h, "k_csi_dir"))) return rc;
  for (int k = 1; k < n_iter; ++k) {
    FwdArgs<T> f = fwd_args<T>(h, alpha);
    if ((rc = launch_fwd<T>(h, f, true))) return rc;
    if ((rc = launch_reduce<T>(h, (const cx<T>*)h->J, (const cx<T>*)h->E, R0))) return rc;
    hipLaunchKernelGGL(k_csi_residual<T>, dim3((NO + 15) / 16, h->B), dim3(256), 0, h->stream,
                       (const cx<T>*)h->Dpart, h->ntiles, (const cx<T>*)h->esca, (cx<T>*)h->dres, NO);
    if ((rc = check_launch(h, "k_csi_residual"))) return rc;
    if ((rc = launch_adj_gemm<T>(h, (const cx<T>*)h->dres, (cx<T>*)h->h))) return rc;
    AdjArgs<T> a = adj_args<T>(h, h->g0, nullptr, nullptr, nullptr, nullptr);
    a.R = R0;
    a.den = nullptr;
    a.gR = nullptr;
    if ((rc = launch_adj<T>(h, a))) return rc;
    hipLaunchKernelGGL(k_sumsq<T>, dim3(h->B), dim3(256), 0, h->stream, (const cx<T>*)h->g0, len, h->gnorm);
    if ((rc = check_launch(h, "k_sumsq"))) return rc;
    hipLaunchKernelGGL(k_csi_dir<T>, dim3(h->B), dim3(256), 0, h->stream, (const cx<T>*)h->g0, p, h->gnorm, gprev,
                       dot, len, 0);
    if ((rc = check_launch(h, "k_csi_dir"))) return rc;
    f.in = p;
    f.einc = nullptr;
    if ((rc = launch_fwd<T>(h, f, true))) return rc;
    if ((rc = launch_reduce<T>(h, (const cx<T>*)h->J, (const cx<T>*)h->E, R0))) return rc;
    hipLaunchKernelGGL(k_csi_step<T>, dim3(h->B), dim3(256), 0, h->stream, h->lsp, (const cx<T>*)h->Dpart,
                       h->ntiles, h->Ni, h->Ns, dot, h->Ss, h->Sd, (const cx<T>*)p, alpha, h->K * h->K);
    if ((rc = check_launch(h, "k_csi_step"))) return rc;
  }
  return PDF_OK;
}

// ------------------------------------------------------------------ several frequencies
//
// A container handle (F > 1, batch 1) holds one handle per frequency.  Per
// frequency: coefficients alpha_f = alpha + f Ni K^2 (the [F][Ni][K][K]
// layout), the forward convolution, the pixel reduction (which also writes its
// per-pixel sums weighted by 1/||E_inc,f||^2 into the container's wsum), the
// data residual, G_S,f^H d_f and the adjoint.  Joint: the contrast R, chi,
// den and lsp (k_mf_combine), the loss and the regulariser gradient
// (the container's regulariser pass, L^Data = sum_f ||d_f||^2 / ||E_sca,f||^2),
// the Adam step count and bias corrections.

// Forward passes of every frequency and the joint contrast; data residual norms per frequency.
template <typename T>
static int mf_forward(pdf_handle* h, const void* alpha) {
  int rc;
  const size_t len = size_t(h->sub[0]->Ni) * h->K * h->K;
  for (int f = 0; f < h->F; ++f) {
    pdf_handle* s = h->sub[f];
    if ((rc = launch_fwd<T>(s, fwd_args<T>(s, (const cx<T>*)alpha + f * len), true))) return fail(h, rc, s->err_msg);
    if ((rc = launch_reduce<T>(s, (const cx<T>*)s->J, (const cx<T>*)s->E, nullptr))) return fail(h, rc, s->err_msg);
  }
  hipLaunchKernelGGL(k_mf_combine<T>, dim3(h->ntiles), dim3(256), 0, h->stream, (const double*)h->wsum, h->F, h->N,
                     h->prm.beta, (const cx<T>*)nullptr, (cx<T>*)h->R, (T*)h->den, (cx<T>*)h->chi, h->lsp);
  if ((rc = check_launch(h, "k_mf_combine"))) return rc;
  for (int f = 0; f < h->F; ++f) {
    pdf_handle* s = h->sub[f];
    const int NO = s->Ni * s->Ns;
    hipLaunchKernelGGL(k_csi_residual<T>, dim3((NO + 15) / 16, 1), dim3(256), 0, h->stream, (const cx<T>*)s->Dpart,
                       s->ntiles, (const cx<T>*)s->esca, (cx<T>*)s->dres, NO);
    hipLaunchKernelGGL(k_sumsq<T>, dim3(1), dim3(256), 0, h->stream, (const cx<T>*)s->dres, size_t(NO), h->dn + f);
  }
  return check_launch(h, "data residuals");
}

template <typename T>
static int run_iteration_mf(pdf_handle* h, const void* alpha, void* grad, double* loss, void* alpha_upd, void* m,
                            void* v, int* tstep, const int* frozen) {
  int rc;
  if ((rc = mf_forward<T>(h, alpha))) return rc;
  if ((rc = launch_reg<T>(h, loss, tstep, frozen))) return rc;
  const size_t len = size_t(h->sub[0]->Ni) * h->K * h->K;
  for (int f = 0; f < h->F; ++f) {
    pdf_handle* s = h->sub[f];
    if ((rc = launch_adj_gemm<T>(s, (const cx<T>*)s->dres, (cx<T>*)s->h))) return fail(h, rc, s->err_msg);
    AdjArgs<T> a = adj_args<T>(s, grad ? (cx<T>*)grad + f * len : nullptr,
                               alpha_upd ? (cx<T>*)alpha_upd + f * len : nullptr, m ? (T*)m + 2 * f * len : nullptr,
                               v ? (T*)v + 2 * f * len : nullptr, frozen);
    a.R = (const cx<T>*)h->R;
    a.den = (const T*)h->den;
    a.gR = (const cx<T>*)h->gR;
    a.adam_c = h->adam_c;
    a.gr_w = T(1.0 / s->ss_host);
    if ((rc = launch_adj<T>(s, a))) return fail(h, rc, s->err_msg);
  }
  return PDF_OK;
}

// Start value over all frequencies (Sec. 3.1 with the frequencies joined): the
// back-propagation currents per frequency, the joint least-squares contrast
// R_0, the gradient of the summed L^CSI at zero per frequency, and one exact
// line-search step along it.
template <typename T>
static int run_init_mf(pdf_handle* h, void* alpha_out) {
  int rc;
  MfPairs<T> pr;
  std::memset(&pr, 0, sizeof(pr));
  pr.F = h->F;
  pr.Ni = h->sub[0]->Ni;
  pr.N = h->N;
  for (int f = 0; f < h->F; ++f) {
    pdf_handle* s = h->sub[f];
    cx<T>* u = (cx<T>*)s->h;
    if ((rc = launch_adj_gemm<T>(s, (const cx<T>*)s->esca, u))) return fail(h, rc, s->err_msg);
    if ((rc = launch_reduce<T>(s, u, u, nullptr))) return fail(h, rc, s->err_msg);
    hipLaunchKernelGGL(k_bp_gamma<T>, dim3(s->Ni), dim3(256), 0, h->stream, (const cx<T>*)s->Dpart, s->ntiles,
                       (const cx<T>*)s->esca, u, s->Ni, s->Ns, s->N);
    FwdArgs<T> fa = fwd_args<T>(s, u);
    fa.J = nullptr;
    fa.beta = T(0);
    if ((rc = launch_fwd<T>(s, fa, false))) return fail(h, rc, s->err_msg);
    pr.J[f] = u;
    pr.E[f] = (const cx<T>*)s->E;
    pr.w[f] = 1.0 / s->ss_host;
  }
  hipLaunchKernelGGL(k_mf_bp_contrast<T>, dim3((h->N + 255) / 256), dim3(256), 0, h->stream, pr, h->prm.beta,
                     (cx<T>*)h->R0);
  if ((rc = check_launch(h, "k_mf_bp_contrast"))) return rc;
  MfLineSearch<T> ls;
  std::memset(&ls, 0, sizeof(ls));
  ls.F = h->F;
  const size_t len = size_t(h->sub[0]->Ni) * h->K * h->K;
  for (int f = 0; f < h->F; ++f) {
    pdf_handle* s = h->sub[f];
    cx<T>* u = (cx<T>*)s->h;
    if ((rc = launch_adj_gemm<T>(s, (const cx<T>*)s->esca, u))) return fail(h, rc, s->err_msg);
    AdjArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.E = (const cx<T>*)s->einc;
    a.e_shared = 1;
    a.h = u;
    a.R = (const cx<T>*)h->R0;
    a.Ss = s->Ss;
    a.Sd = s->Sd;
    a.hsign = -1.0;
    a.ghat = (const cx<T>*)s->ghat;
    a.tw = (const cx<T>*)s->tw;
    a.galpha = (cx<T>*)s->g0;
    a.gr_w = T(1);
    a.Ni = s->Ni;
    a.K = s->K;
    a.beta = T(s->prm.beta);
    if ((rc = launch_adj<T>(s, a))) return fail(h, rc, s->err_msg);
    hipLaunchKernelGGL(k_sumsq<T>, dim3(1), dim3(256), 0, h->stream, (const cx<T>*)s->g0, len, h->gn + f);
    // curvature along g_f with R_0: A_d g = G_S,f J_g, A_s g = R_0 (G_D J_g + beta J_g) - beta J_g
    FwdArgs<T> fa = fwd_args<T>(s, s->g0);
    fa.einc = nullptr;
    if ((rc = launch_fwd<T>(s, fa, true))) return fail(h, rc, s->err_msg);
    if ((rc = launch_reduce<T>(s, (const cx<T>*)s->J, (const cx<T>*)s->E, (const cx<T>*)h->R0)))
      return fail(h, rc, s->err_msg);
    const int NO = s->Ni * s->Ns, ndp = (NO + 15) / 16;
    hipLaunchKernelGGL(k_mf_dnorm<T>, dim3(ndp), dim3(256), 0, h->stream, (const cx<T>*)s->Dpart, s->ntiles, NO,
                       h->mf_dp + size_t(f) * ndp);
    ls.dpart[f] = h->mf_dp + size_t(f) * ndp;
    ls.ndp = ndp;
    ls.lsp[f] = s->lsp;
    ls.Sd[f] = s->Sd;
    ls.Ss[f] = s->Ss;
    ls.g0[f] = (const cx<T>*)s->g0;
  }
  ls.gn = h->gn;
  ls.alpha = (cx<T>*)alpha_out;
  ls.ntiles = h->sub[0]->ntiles;
  ls.len = int(len);
  hipLaunchKernelGGL(k_mf_line_search<T>, dim3(1), dim3(256), 0, h->stream, ls);
  return check_launch(h, "k_mf_line_search");
}

// ------------------------------------------------------------------ setup

template <typename T>
static int upload(pdf_handle* h, void** dst, const std::vector<std::complex<double>>& src, double scale) {
  std::vector<cx<T>> tmp(src.size());
  for (size_t i = 0; i < src.size(); ++i) tmp[i] = cx<T>{T(src[i].real() * scale), T(src[i].imag() * scale)};
  HIP_TRY(hipMalloc(dst, sizeof(cx<T>) * tmp.size()));
  HIP_TRY(hipMemcpy(*dst, tmp.data(), sizeof(cx<T>) * tmp.size(), hipMemcpyHostToDevice));
  return PDF_OK;
}

template <typename T>
static int setup_impl(pdf_handle* h, const pdfh::Tables& t) {
  int rc;
  const double inv = 1.0 / (double(h->P) * h->P);
  if ((rc = upload<T>(h, &h->ghat, t.ghat, inv))) return rc;
  // the P twiddles exp(-2 pi i k / P), then the half-shift values
  // hs[m] = 2 / (1 - exp(-i pi (2m + 1) / M)) of the compact tile's row products over two
  // periods from m = -M/2
  std::vector<std::complex<double>> tw(h->P + 2 * h->M);
  for (int k = 0; k < h->P; ++k) tw[k] = std::polar(1.0, -2.0 * M_PI * k / h->P);
  for (int p = 0; p < 2 * h->M; ++p) {
    const int m = (p + h->M - h->M / 2) % h->M;   // (p - M/2) mod M
    tw[h->P + p] = 2.0 / (1.0 - std::polar(1.0, -M_PI * (2.0 * m + 1.0) / h->M));
  }
  if ((rc = upload<T>(h, &h->tw, tw, 1.0))) return rc;
  if ((rc = upload<T>(h, &h->gs, t.gs, 1.0))) return rc;
  {
    std::vector<std::complex<double>> gst(t.gs.size());
    for (int q = 0; q < h->Ns; ++q)
      for (int n = 0; n < h->N; ++n) gst[size_t(n) * h->Ns + q] = t.gs[size_t(q) * h->N + n];
    if ((rc = upload<T>(h, &h->gsT, gst, 1.0))) return rc;
  }
  if (sizeof(T) == 4 && h->N % 32 == 0) {
    // A operands of the FP32 receiver GEMM (real-expanded 32x32x2 MFMA) in lane
    // order: for pixel n and row tile r, lane m + 32 cp holds sgn * part of
    // G_S[q][n], q = 16 r + m / 2, part = (m % 2) ^ cp (0 Re, 1 Im), sgn = -1
    // for (m % 2, cp) = (0, 1); zero for q >= Ns
    const int nrt = (h->Ns + 15) / 16;
    std::vector<float> ga(size_t(h->N) * nrt * 64);
    for (int n = 0; n < h->N; ++n)
      for (int r = 0; r < nrt; ++r)
        for (int l = 0; l < 64; ++l) {
          const int m = l & 31, cp = l >> 5, c = m & 1, part = c ^ cp, q = 16 * r + (m >> 1);
          float v = 0.f;
          if (q < h->Ns) {
            const std::complex<double>& g = t.gs[size_t(q) * h->N + n];
            v = float(part ? g.imag() : g.real());
            if (c == 0 && cp == 1) v = -v;
          }
          ga[(size_t(n) * nrt + r) * 64 + l] = v;
        }
    HIP_TRY(hipMalloc(&h->gsA, sizeof(float) * ga.size()));
    HIP_TRY(hipMemcpy(h->gsA, ga.data(), sizeof(float) * ga.size(), hipMemcpyHostToDevice));
  }
  if ((rc = upload<T>(h, &h->einc, t.einc, 1.0))) return rc;
  // ||E_inc||^2 of the values actually used (after rounding to T)
  double ss = 0.0;
  for (auto& z : t.einc) {
    const double re = double(T(z.real())), im = double(T(z.imag()));
    ss += re * re + im * im;
  }
  if (!(ss > 0.0)) return fail(h, PDF_ENONFINITE, "||E_inc|| = 0");
  HIP_TRY(hipMalloc(&h->Ss, sizeof(double)));
  HIP_TRY(hipMemcpy(h->Ss, &ss, sizeof(double), hipMemcpyHostToDevice));
  h->ss_host = ss;
  const size_t C = sizeof(cx<T>);
  const size_t B = h->B, Ni = h->Ni, Ns = h->Ns, N = h->N, KK = size_t(h->K) * h->K;
  HIP_TRY(hipMalloc(&h->Sd, sizeof(double) * B));
  HIP_TRY(hipMalloc(&h->esca, C * B * Ni * Ns));
  HIP_TRY(hipMalloc(&h->J, C * B * Ni * N));
  HIP_TRY(hipMalloc(&h->E, C * B * Ni * N));
  HIP_TRY(hipMalloc(&h->h, C * B * Ni * N));
  HIP_TRY(hipMalloc(&h->R, C * B * N));
  HIP_TRY(hipMalloc(&h->den, sizeof(T) * B * N));
  HIP_TRY(hipMalloc(&h->chi, C * B * N));
  HIP_TRY(hipMalloc(&h->gR, C * B * N));
  HIP_TRY(hipMalloc(&h->R0, C * B * N));
  HIP_TRY(hipMalloc(&h->Dpart, C * B * h->ntiles * Ni * Ns));
  HIP_TRY(hipMalloc(&h->dres, C * B * Ni * Ns));
  HIP_TRY(hipMalloc(&h->lsp, sizeof(double) * B * h->ntiles));
  HIP_TRY(hipMalloc(&h->g0, C * B * Ni * KK));
  HIP_TRY(hipMalloc(&h->gnorm, sizeof(double) * B));
  HIP_TRY(hipMalloc(&h->err, sizeof(double) * B));
  HIP_TRY(hipMalloc(&h->frozen, sizeof(int) * B));
  HIP_TRY(hipMalloc(&h->tstep, sizeof(int) * B));
  HIP_TRY(hipMalloc(&h->adam_c, 2 * sizeof(double) * B));
  HIP_TRY(hipMalloc(&h->m, 2 * sizeof(T) * B * Ni * KK));
  HIP_TRY(hipMalloc(&h->v, 2 * sizeof(T) * B * Ni * KK));
  HIP_TRY(hipMalloc(&h->loss, sizeof(double) * 8 * B));
  HIP_TRY(hipMalloc(&h->loss_w, sizeof(double) * 8 * B));
  if (h->big) {
    HIP_TRY(hipMalloc(&h->S, C * B * Ni * N * 2));
    HIP_TRY(hipMalloc(&h->GJ, C * B * Ni * N));
    const size_t nblk = (N + 255) / 256;
    HIP_TRY(hipMalloc(&h->big_ws, sizeof(T) * B * 4 * N + sizeof(double) * B * nblk * 2));
    HIP_TRY(hipMalloc(&h->reg_part, sizeof(double) * B * nblk * 6));
  }
  if (h->prm.cco_in_loss) {
    HIP_TRY(hipMalloc(&h->ccl_ws, sizeof(T) * B * kCclArrays * N));
    HIP_TRY(hipMalloc(&h->chic, sizeof(cx<T>) * B * N));
    HIP_TRY(hipMalloc(&h->Rc, sizeof(cx<T>) * B * N));
    HIP_TRY(hipMalloc(&h->ccl_part, sizeof(double) * B * ((N + 255) / 256)));
  }
  return PDF_OK;
}

static int check_geometry(const pdf_grid* grid, double freq, const pdf_array* tx, const pdf_array* rx) {
  if (!grid || !tx || !rx || !tx->xy || !rx->xy) return fail(nullptr, PDF_EINVAL, "null argument");
  if (grid->M < 1 || !(grid->side > 0) || !std::isfinite(grid->side) || !(freq > 0) || !std::isfinite(freq))
    return fail(nullptr, PDF_EINVAL, "invalid grid or frequency");
  if (tx->n < 1 || rx->n < 1) return fail(nullptr, PDF_EINVAL, "need at least one transmitter and one receiver");
  for (int i = 0; i < 2 * tx->n; ++i)
    if (!std::isfinite(tx->xy[i])) return fail(nullptr, PDF_EINVAL, "non-finite transmitter position");
  for (int i = 0; i < 2 * rx->n; ++i)
    if (!std::isfinite(rx->xy[i])) return fail(nullptr, PDF_EINVAL, "non-finite receiver position");
  return PDF_OK;
}

extern "C" int pdf_tables_host(const pdf_grid* grid, double freq_hz, const pdf_array* tx, const pdf_array* rx,
                               double* ghat, double* gs, double* einc) {
  int rc = check_geometry(grid, freq_hz, tx, rx);
  if (rc) return rc;
  pdfh::Geometry g{grid->M, grid->side, grid->cx, grid->cy, freq_hz, tx->n, rx->n, tx->xy, rx->xy};
  pdfh::Tables t;
  t.want_ghat = ghat != nullptr;
  t.want_gs = gs != nullptr;
  t.want_einc = einc != nullptr;
  std::string err;
  if (pdfh::build_tables(g, &t, &err)) return fail(nullptr, PDF_EINVAL, err);
  if (ghat) std::memcpy(ghat, t.ghat.data(), t.ghat.size() * sizeof(std::complex<double>));
  if (gs) std::memcpy(gs, t.gs.data(), t.gs.size() * sizeof(std::complex<double>));
  if (einc) std::memcpy(einc, t.einc.data(), t.einc.size() * sizeof(std::complex<double>));
  return PDF_OK;
}

extern "C" int pdf_timing(pdf_handle* h, int32_t enable, int32_t max_steps) {
  if (!h) return fail(h, PDF_EINVAL, "null handle");
  if (h->F > 1) return fail(h, PDF_EUNSUPPORTED, "per-kernel timing covers single-frequency handles");
  h->timing = false;
  h->ev_used = 0;
  if (!enable) return PDF_OK;
  if (max_steps < 1 || max_steps > 100000) return fail(h, PDF_EINVAL, "max_steps out of range");
  const size_t need = size_t(max_steps) * (PDF_NKERNELS + 1);
  while (h->events.size() < need) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    h->events.push_back(e);
  }
  h->timing_max = max_steps;
  h->timing = true;
  return PDF_OK;
}

extern "C" int pdf_timing_read(pdf_handle* h, double* avg_ms, int32_t* n_steps) {
  if (!h || !avg_ms || !n_steps) return fail(h, PDF_EINVAL, "null argument");
  HIP_TRY(hipStreamSynchronize(h->stream));
  const int per_step = PDF_NKERNELS + 1;
  const int steps = h->ev_used / per_step;
  for (int k = 0; k < PDF_NKERNELS; ++k) avg_ms[k] = 0.0;
  for (int s = 0; s < steps; ++s)
    for (int k = 0; k < PDF_NKERNELS; ++k) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, h->events[s * per_step + k], h->events[s * per_step + k + 1]));
      avg_ms[k] += ms;
    }
  for (int k = 0; k < PDF_NKERNELS; ++k) avg_ms[k] = steps ? avg_ms[k] / steps : 0.0;
  *n_steps = steps;
  return PDF_OK;
}

extern "C" void pdf_destroy(pdf_handle* h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (pdf_handle*& s : h->sub) {
    pdf_destroy(s);
    s = nullptr;
  }
  for (void* p : {(void*)h->wsum, (void*)h->dn, (void*)h->gn, (void*)h->sdf, (void*)h->mf_dp})
    if (p) (void)hipFree(p);
  for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
  void* ptrs[] = {h->gsT, h->gsA, h->ghat, h->tw,   h->gs,   h->einc, h->Ss,    h->Sd,     h->esca,   h->J,
                  h->E,    h->h,    h->R,    h->den,  h->chi,   h->gR,     h->Dpart,  h->dres,
                  h->lsp,  h->R0,   h->g0,   h->gnorm, h->err,  h->frozen, h->tstep,  h->m,
                  h->v,    h->loss, h->loss_w, h->adam_c, h->fc_ws, h->csi_ws, h->S,     h->GJ,
                  h->big_ws, h->ccl_ws, h->chic, h->Rc, h->ccl_part, h->reg_part};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete h;
}

extern "C" int pdf_setup(const pdf_grid* grid, double freq_hz, const pdf_array* tx, const pdf_array* rx, int32_t K,
                         int32_t batch, const pdf_params* params, void* stream, pdf_handle** out) {
  if (!out) return fail(nullptr, PDF_EINVAL, "out is null");
  *out = nullptr;
  int rc = check_geometry(grid, freq_hz, tx, rx);
  if (rc) return rc;
  pdf_params prm;
  if (params) {
    if (params->version == PDF_PARAMS_VERSION) {
      prm = *params;
    } else if (params->version == 1) {  // the version-1 struct ends before cco_in_loss
      pdf_default_params(&prm);
      std::memcpy(&prm, params, offsetof(pdf_params, cco_in_loss));
      prm.version = PDF_PARAMS_VERSION;
    } else {
      return fail(nullptr, PDF_EINVAL, "pdf_params version mismatch");
    }
  } else {
    pdf_default_params(&prm);
  }
  if (prm.precision != PDF_FP32 && prm.precision != PDF_FP64) return fail(nullptr, PDF_EINVAL, "bad precision");
  if (K < 1 || K > grid->M) return fail(nullptr, PDF_EINVAL, "K must satisfy 1 <= K <= M");
  if (batch < 1) return fail(nullptr, PDF_EINVAL, "batch must be >= 1");
  if (!stream) return fail(nullptr, PDF_EINVAL, "a non-default stream is required");
  if (!supported_m(prm.precision, grid->M))
    return fail(nullptr, PDF_EUNSUPPORTED, "M must be 8, 16, 32, 48, 64, 96, 128 or 256");
  if (rx->n > 64) return fail(nullptr, PDF_EUNSUPPORTED, "at most 64 receivers");
  if (!(prm.beta > 0) || prm.gf_radius < 0) return fail(nullptr, PDF_EINVAL, "beta must be > 0");
  if (prm.cco_in_loss != 0 && prm.cco_in_loss != 1) return fail(nullptr, PDF_EINVAL, "cco_in_loss must be 0 or 1");
  if (prm.cco_in_loss && big_grid(prm.precision, grid->M))
    return fail(nullptr, PDF_EUNSUPPORTED, "the loss on the CCO image covers the LDS-resident grids");
  pdf_handle* h = new pdf_handle();
  h->prec = prm.precision;
  h->prm = prm;
  h->M = grid->M;
  h->N = grid->M * grid->M;
  h->P = 2 * grid->M;
  h->K = K;
  h->Ni = tx->n;
  h->Ns = rx->n;
  h->B = batch;
  h->big = big_grid(prm.precision, grid->M);
  h->stream = (hipStream_t)stream;
  // the handle's device and its copy of the static scratch (looked up here, at
  // set-up, with that device current; a failure only disables the entry
  // points that use it, which then report it)
  if (hipGetDevice(&h->device) == hipSuccess) {
    const hipError_t se = scratch_address(h->device, &h->scratch_dev);
    if (se != hipSuccess) h->scratch_err = std::string("hipGetSymbolAddress: ") + hipGetErrorString(se);
  } else {
    h->scratch_err = "hipGetDevice failed";
  }
  const size_t csz = prm.precision == PDF_FP32 ? 8 : 16;
  int tile = 256;
  if (prm.precision == PDF_FP32 && h->Ni > 64) {
    delete h;
    return fail(nullptr, PDF_EUNSUPPORTED, "at most 64 incidences");
  }
  // the FP64 reduction stages [Ni][tile] currents in LDS; the FP32 one has a fixed
  // 256-pixel tile staged in 128-pixel halves (any Ni <= 64)
  while (prm.precision == PDF_FP64 && tile > 64 && size_t(h->Ni) * tile * csz > 64 * 1024) tile >>= 1;
  if (prm.precision == PDF_FP64 && size_t(h->Ni) * tile * csz > 64 * 1024) {
    delete h;
    return fail(nullptr, PDF_EUNSUPPORTED, "too many incidences for the pixel-reduction tile");
  }
  h->tile = tile;
  h->ntiles = (h->N + tile - 1) / tile;
  pdfh::Geometry g{grid->M, grid->side, grid->cx, grid->cy, freq_hz, tx->n, rx->n, tx->xy, rx->xy};
  pdfh::Tables t;
  std::string err;
  if (pdfh::build_tables(g, &t, &err)) {
    delete h;
    return fail(nullptr, PDF_EINVAL, err);
  }
  rc = prm.precision == PDF_FP32 ? setup_impl<float>(h, t) : setup_impl<double>(h, t);
  if (rc) {
    g_last_error = h->err_msg;
    pdf_destroy(h);
    return rc;
  }
  *out = h;
  return PDF_OK;
}

// Container buffers of a handle over several frequencies (see mf_forward).
template <typename T>
static int setup_mf_buffers(pdf_handle* h) {
  const size_t C = sizeof(cx<T>), N = h->N, KK = size_t(h->K) * h->K, len = size_t(h->Ni) * KK;
  HIP_TRY(hipMalloc(&h->R, C * N));
  HIP_TRY(hipMalloc(&h->den, sizeof(T) * N));
  HIP_TRY(hipMalloc(&h->chi, C * N));
  HIP_TRY(hipMalloc(&h->gR, C * N));
  HIP_TRY(hipMalloc(&h->R0, C * N));
  HIP_TRY(hipMalloc(&h->lsp, sizeof(double) * h->ntiles));
  HIP_TRY(hipMalloc(&h->Ss, sizeof(double)));
  const double one = 1.0;  // the joint state loss comes weighted by 1 / ||E_inc,f||^2 already
  HIP_TRY(hipMemcpy(h->Ss, &one, sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(hipMalloc(&h->loss, sizeof(double) * 8));
  HIP_TRY(hipMalloc(&h->loss_w, sizeof(double) * 8));
  HIP_TRY(hipMalloc(&h->tstep, sizeof(int)));
  HIP_TRY(hipMalloc(&h->frozen, sizeof(int)));
  HIP_TRY(hipMalloc(&h->adam_c, 2 * sizeof(double)));
  HIP_TRY(hipMalloc(&h->err, sizeof(double)));
  HIP_TRY(hipMalloc(&h->m, 2 * sizeof(T) * len));
  HIP_TRY(hipMalloc(&h->v, 2 * sizeof(T) * len));
  HIP_TRY(hipMalloc(&h->wsum, sizeof(double) * 4 * N * h->F));
  HIP_TRY(hipMalloc(&h->dn, sizeof(double) * h->F));
  HIP_TRY(hipMalloc(&h->gn, sizeof(double) * h->F));
  HIP_TRY(hipMalloc(&h->sdf, sizeof(double) * h->F));
  HIP_TRY(hipMalloc(&h->mf_dp, sizeof(double) * h->F * ((h->sub[0]->Ni * h->Ns + 15) / 16)));
  if (h->big) {
    HIP_TRY(hipMalloc(&h->big_ws, sizeof(T) * 4 * N + sizeof(double) * ((N + 255) / 256) * 2));
    HIP_TRY(hipMalloc(&h->reg_part, sizeof(double) * ((N + 255) / 256) * 6));
  }
  return PDF_OK;
}

extern "C" int pdf_setup_freq(const pdf_grid* grid, const pdf_freq* freq, const pdf_array* tx, const pdf_array* rx,
                              int32_t K, int32_t batch, const pdf_params* params, void* stream, pdf_handle** out) {
  if (!out) return fail(nullptr, PDF_EINVAL, "out is null");
  *out = nullptr;
  if (!freq || !freq->hz || freq->n_freq < 1 || freq->n_freq > kMaxFreq)
    return fail(nullptr, PDF_EINVAL, "pdf_freq needs 1 to 8 frequencies");
  if (freq->n_freq == 1) return pdf_setup(grid, freq->hz[0], tx, rx, K, batch, params, stream, out);
  if (batch != 1)
    return fail(nullptr, PDF_EUNSUPPORTED, "several frequencies: one reconstruction per handle (batch 1)");
  if (params && params->version == PDF_PARAMS_VERSION && params->cco_in_loss)
    return fail(nullptr, PDF_EUNSUPPORTED, "the loss on the CCO image covers single-frequency handles");
  pdf_handle* h = new pdf_handle();
  h->F = freq->n_freq;
  for (int f = 0; f < h->F; ++f) {
    const int rc = pdf_setup(grid, freq->hz[f], tx, rx, K, 1, params, stream, &h->sub[f]);
    if (rc) {
      const std::string msg = g_last_error;
      pdf_destroy(h);
      return fail(nullptr, rc, "frequency " + std::to_string(f) + ": " + msg);
    }
  }
  const pdf_handle* s0 = h->sub[0];
  h->prec = s0->prec;
  h->prm = s0->prm;
  h->M = s0->M;
  h->N = s0->N;
  h->P = s0->P;
  h->K = s0->K;
  h->Ns = s0->Ns;
  h->Ni = h->F * s0->Ni;
  h->B = 1;
  h->big = s0->big;
  h->stream = s0->stream;
  h->device = s0->device;
  h->scratch_dev = s0->scratch_dev;
  h->scratch_err = s0->scratch_err;
  h->tile = 256;
  h->ntiles = (h->N + 255) / 256;
  const int rc = h->prec == PDF_FP32 ? setup_mf_buffers<float>(h) : setup_mf_buffers<double>(h);
  if (rc) {
    g_last_error = h->err_msg;
    pdf_destroy(h);
    return rc;
  }
  for (int f = 0; f < h->F; ++f) {
    h->sub[f]->mf_wsum = h->wsum + size_t(f) * 4 * h->N;
    h->sub[f]->mf_w = 1.0 / h->sub[f]->ss_host;
  }
  *out = h;
  return PDF_OK;
}

extern "C" int pdf_set_data(pdf_handle* h, const void* esca_dev) {
  if (!h || !esca_dev) return fail(h, PDF_EINVAL, "null argument");
  if (h->F > 1) {
    const size_t csz = h->prec == PDF_FP32 ? 8 : 16;
    const size_t per = size_t(h->sub[0]->Ni) * h->Ns * csz;
    for (int f = 0; f < h->F; ++f) {
      if (int rc = pdf_set_data(h->sub[f], static_cast<const char*>(esca_dev) + f * per))
        return fail(h, rc, "frequency " + std::to_string(f) + ": " + h->sub[f]->err_msg);
      HIP_TRY(hipMemcpyAsync(h->sdf + f, h->sub[f]->Sd, sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    }
    h->data_set = true;
    return PDF_OK;
  }
  const size_t csz = h->prec == PDF_FP32 ? 8 : 16;
  HIP_TRY(hipMemcpyAsync(h->esca, esca_dev, csz * size_t(h->B) * h->Ni * h->Ns, hipMemcpyDeviceToDevice,
                         h->stream));
  const size_t len = size_t(h->Ni) * h->Ns;
  if (h->prec == PDF_FP32)
    hipLaunchKernelGGL(k_sumsq<float>, dim3(h->B), dim3(256), 0, h->stream, (const cx<float>*)h->esca, len, h->Sd);
  else
    hipLaunchKernelGGL(k_sumsq<double>, dim3(h->B), dim3(256), 0, h->stream, (const cx<double>*)h->esca, len,
                       h->Sd);
  int rc = check_launch(h, "k_sumsq");
  if (rc) return rc;
  std::vector<double> sd(h->B);
  HIP_TRY(hipMemcpyAsync(sd.data(), h->Sd, sizeof(double) * h->B, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  for (double s : sd)
    if (!(s > 0.0) || !std::isfinite(s)) return fail(h, PDF_ENONFINITE, "||E_sca|| = 0 or not finite");
  h->data_set = true;
  return PDF_OK;
}

extern "C" int pdf_loss_grad(pdf_handle* h, const void* alpha_dev, void* grad_dev, double* loss_dev) {
  if (!h || !alpha_dev) return fail(h, PDF_EINVAL, "null argument");
  if (!h->data_set) return fail(h, PDF_EINVAL, "pdf_set_data has not been called");
  // without a gradient output only the forward kernels and the loss pass run
  if (!grad_dev)
    return h->prec == PDF_FP32 ? run_loss<float>(h, alpha_dev, loss_dev) : run_loss<double>(h, alpha_dev, loss_dev);
  return h->prec == PDF_FP32
             ? run_iteration<float>(h, alpha_dev, grad_dev, loss_dev, nullptr, nullptr, nullptr, nullptr, nullptr)
             : run_iteration<double>(h, alpha_dev, grad_dev, loss_dev, nullptr, nullptr, nullptr, nullptr, nullptr);
}

extern "C" int pdf_step(pdf_handle* h, void* alpha_dev, void* m_dev, void* v_dev, int32_t* t_dev,
                        double* loss_dev) {
  if (!h || !alpha_dev || !m_dev || !v_dev || !t_dev) return fail(h, PDF_EINVAL, "null argument");
  if (!h->data_set) return fail(h, PDF_EINVAL, "pdf_set_data has not been called");
  return h->prec == PDF_FP32
             ? run_iteration<float>(h, alpha_dev, nullptr, loss_dev, alpha_dev, m_dev, v_dev, t_dev, nullptr)
             : run_iteration<double>(h, alpha_dev, nullptr, loss_dev, alpha_dev, m_dev, v_dev, t_dev, nullptr);
}

extern "C" int pdf_init_alpha_csi(pdf_handle* h, int32_t n_iter, void* alpha_dev) {
  if (!h || !alpha_dev) return fail(h, PDF_EINVAL, "null argument");
  if (h->F > 1) return fail(h, PDF_EUNSUPPORTED, "the full CSI start covers single-frequency handles");
  if (n_iter < 1) return fail(h, PDF_EINVAL, "n_iter must be at least 1");
  if (!h->data_set) return fail(h, PDF_EINVAL, "pdf_set_data has not been called");
  const size_t need = csi_workspace_bytes(h);
  if (n_iter > 1 && h->csi_bytes < need) {
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (h->csi_ws) HIP_TRY(hipFree(h->csi_ws));
    h->csi_ws = nullptr;
    h->csi_bytes = 0;
    HIP_TRY(hipMalloc(&h->csi_ws, need));
    h->csi_bytes = need;
  }
  return h->prec == PDF_FP32 ? run_csi<float>(h, n_iter, alpha_dev, h->csi_ws)
                             : run_csi<double>(h, n_iter, alpha_dev, h->csi_ws);
}

extern "C" int pdf_init_alpha_csi_noalloc(pdf_handle* h, int32_t n_iter, void* alpha_dev) {
  if (!h || !alpha_dev) return fail(h, PDF_EINVAL, "null argument");
  if (h->F > 1) return fail(h, PDF_EUNSUPPORTED, "the full CSI start covers single-frequency handles");
  if (n_iter < 1) return fail(h, PDF_EINVAL, "n_iter must be at least 1");
  if (!h->data_set) return fail(h, PDF_EINVAL, "pdf_set_data has not been called");
  const size_t need = csi_workspace_bytes(h);
  if (n_iter > 1 && need > PDF_STATIC_SCRATCH_BYTES)
    return fail(h, PDF_EINVAL,
                "the CSI workspace needs " + std::to_string(need) + " bytes; the static scratch holds " +
                    std::to_string(size_t(PDF_STATIC_SCRATCH_BYTES)) + " (B Ni K^2 too large)");
  if (!h->scratch_dev)
    return fail(h, PDF_EHIP, "the static scratch of this device has no address: " + h->scratch_err);
  return h->prec == PDF_FP32 ? run_csi<float>(h, n_iter, alpha_dev, h->scratch_dev)
                             : run_csi<double>(h, n_iter, alpha_dev, h->scratch_dev);
}

extern "C" int pdf_init_alpha(pdf_handle* h, void* alpha_dev) {
  if (!h || !alpha_dev) return fail(h, PDF_EINVAL, "null argument");
  if (!h->data_set) return fail(h, PDF_EINVAL, "pdf_set_data has not been called");
  return h->prec == PDF_FP32 ? run_init<float>(h, alpha_dev) : run_init<double>(h, alpha_dev);
}

// The linear pieces of the loss applied alone (see pdf_apply), with the
// kernels of the loss-gradient pass: the forward convolution kernel without
// incident field and with beta = 0, the adjoint convolution kernel with R and
// the data term chosen so that its g_J is exactly the input (R = 0) or its g_E
// is (R = 1, zero data term, unit weights), the split-K receiver GEMM with its
// fixed-order sum, and the G_S^H GEMM.
template <typename T>
static int run_apply(pdf_handle* h, int op, const void* x, void* y) {
  int rc;
  const size_t nb = size_t(h->B), npix = nb * h->N;
  auto fill = [&](void* buf, size_t n, double re) -> int {
    hipLaunchKernelGGL(k_fill_cx<T>, dim3((n + 255) / 256), dim3(256), 0, h->stream, (cx<T>*)buf, T(re), T(0), n);
    return check_launch(h, "k_fill_cx");
  };
  if (op == PDF_OP_SYNTH || op == PDF_OP_GD || op == PDF_OP_GD_SYNTH) {
    FwdArgs<T> f = fwd_args<T>(h, x);
    f.einc = nullptr;
    f.beta = T(0);
    if (op == PDF_OP_SYNTH) {
      f.J = (cx<T>*)y;
      f.E = (cx<T>*)h->E;
    } else {
      f.J = op == PDF_OP_GD ? nullptr : (cx<T>*)h->J;
      f.E = (cx<T>*)y;
    }
    return launch_fwd<T>(h, f, op != PDF_OP_GD);
  }
  if (op == PDF_OP_SYNTH_ADJ || op == PDF_OP_GD_SYNTH_ADJ) {
    // unit weights: 2 / Ss = 2 hsign / Sd = 1
    hipLaunchKernelGGL(k_fill_double, dim3((h->B + 255) / 256), dim3(256), 0, h->stream, h->gnorm, 2.0, h->B);
    if ((rc = check_launch(h, "k_fill_double"))) return rc;
    AdjArgs<T> a = adj_args<T>(h, y, nullptr, nullptr, nullptr, nullptr);
    a.J = nullptr;
    a.gR = nullptr;
    a.den = nullptr;
    a.Ss = h->gnorm;
    a.Sd = h->gnorm;
    a.hsign = 1.0;
    a.E = (const cx<T>*)x;
    if (op == PDF_OP_SYNTH_ADJ) {
      // R = 0: g_E = 0, g_J = h = x, result B^H x
      if ((rc = fill(h->R, npix, 0.0))) return rc;
      a.h = (const cx<T>*)x;
    } else {
      // R = 1, h = 0: g_E = x, g_J = -beta x + beta x = 0, result B^H G_D^H x
      if ((rc = fill(h->R, npix, 1.0))) return rc;
      if ((rc = fill(h->h, npix * h->Ni, 0.0))) return rc;
      a.h = (const cx<T>*)h->h;
    }
    return launch_adj<T>(h, a);
  }
  if (op == PDF_OP_GS) {
    if ((rc = fill(h->R, npix, 0.0))) return rc;
    if ((rc = fill(h->dres, nb * h->Ni * h->Ns, 0.0))) return rc;
    if ((rc = launch_reduce<T>(h, (const cx<T>*)x, (const cx<T>*)x, (const cx<T>*)h->R))) return rc;
    const int NO = h->Ni * h->Ns;
    hipLaunchKernelGGL(k_csi_residual<T>, dim3((NO + 15) / 16, h->B), dim3(256), 0, h->stream,
                       (const cx<T>*)h->Dpart, h->ntiles, (const cx<T>*)h->dres, (cx<T>*)y, NO);
    return check_launch(h, "k_csi_residual");
  }
  if (op == PDF_OP_GS_ADJ) return launch_adj_gemm<T>(h, (const cx<T>*)x, (cx<T>*)y);
  return fail(h, PDF_EINVAL, "unknown operator");
}

extern "C" int pdf_apply(pdf_handle* h, int32_t op, const void* x_dev, void* y_dev) {
  if (!h || !x_dev || !y_dev) return fail(h, PDF_EINVAL, "null argument");
  if (h->F > 1) return fail(h, PDF_EUNSUPPORTED, "the linear pieces are per frequency: apply them to one frequency");
  if (op < PDF_OP_SYNTH || op > PDF_OP_GS_ADJ) return fail(h, PDF_EINVAL, "unknown operator");
  if (x_dev == y_dev) return fail(h, PDF_EINVAL, "x and y must not alias");
  return h->prec == PDF_FP32 ? run_apply<float>(h, op, x_dev, y_dev) : run_apply<double>(h, op, x_dev, y_dev);
}

// (1/n) sum x^2 of n reals in one workgroup (fixed order, FP64 accumulation).
template <typename T>
__global__ __launch_bounds__(1024) void k_mean_square(const T* x, int64_t n, double* out) {
  __shared__ double red[16];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += double(x[i]) * double(x[i]);
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) out[0] = s / double(n);
}

extern "C" int pdf_mean_square(int32_t precision, int64_t n, const void* x_dev, double* out_dev, void* stream) {
  if (!x_dev || !out_dev) return fail(nullptr, PDF_EINVAL, "null argument");
  if (n < 1 || (precision != PDF_FP32 && precision != PDF_FP64))
    return fail(nullptr, PDF_EINVAL, "n must be >= 1 and precision PDF_FP32 or PDF_FP64");
  hipStream_t st = (hipStream_t)stream;
  if (precision == PDF_FP32)
    hipLaunchKernelGGL(k_mean_square<float>, dim3(1), dim3(1024), 0, st, (const float*)x_dev, n, out_dev);
  else
    hipLaunchKernelGGL(k_mean_square<double>, dim3(1), dim3(1024), 0, st, (const double*)x_dev, n, out_dev);
  return check_launch(nullptr, "k_mean_square");
}

// Average duration (ms) of `reps` launches of fn on the handle's stream.
template <class F>
static int time_launches(pdf_handle* h, int reps, F fn, double* ms) {
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(h, PDF_EHIP, "hipEventCreate");
  }
  int rc = fn();  // warm-up (and first-launch set-up) outside the timed range
  if (!rc && hipEventRecord(e0, h->stream) != hipSuccess) rc = fail(h, PDF_EHIP, "hipEventRecord");
  for (int i = 0; i < reps && !rc; ++i) rc = fn();
  float t = 0.f;
  if (!rc && (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
              hipEventElapsedTime(&t, e0, e1) != hipSuccess))
    rc = fail(h, PDF_EHIP, "event timing failed");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = double(t) / reps;
  return rc;
}

// Whether an FP32 handle's grid has the second convolution plan (all 2M rows
// of the padded tile in one CU's LDS).
template <int M>
static bool full_tile_fits() {
  return ConvCfg<float, M>::lds(true) <= 160 * 1024;
}
static bool full_tile_fits(int M) {
  switch (M) {
    case 8: return full_tile_fits<8>();
    case 16: return full_tile_fits<16>();
    case 32: return full_tile_fits<32>();
    case 48: return full_tile_fits<48>();
    case 64: return full_tile_fits<64>();
  }
  return false;
}

extern "C" int pdf_autotune(pdf_handle* h, int32_t reps, int32_t* choice, double* ms) {
  if (!h || reps < 1) return fail(h, PDF_EINVAL, "bad argument");
  if (h->F > 1) {  // the frequency handles share one shape: tune the first, use its choice for all
    if (int rc = pdf_autotune(h->sub[0], reps, choice, ms)) return fail(h, rc, h->sub[0]->err_msg);
    const pdf_handle* s0 = h->sub[0];
    for (int f = 1; f < h->F; ++f) pdf_set_tiles(h->sub[f], s0->tune_ct, s0->tune_pb, s0->tune_fpp, s0->tune_app);
    h->tuned = true;
    return PDF_OK;
  }
  if (h->prec != PDF_FP32 || h->N % 32 != 0) {  // only FP32 handles have choices
    h->tuned = true;
    if (choice) choice[0] = h->tune_ct, choice[1] = h->tune_pb, choice[2] = h->tune_fpp, choice[3] = h->tune_app;
    return PDF_OK;
  }
  int rc;
  double t[9];
  const int cts[3] = {1, 2, 4}, pbs[2] = {4, 8};
  int best_ct = h->tune_ct, best_pb = h->tune_pb;
  for (int i = 0; i < 3; ++i) {
    h->tune_ct = cts[i];
    if ((rc = time_launches(h, reps, [&]() { return launch_adj_gemm<float>(h, (const cx<float>*)h->dres,
                                                                           (cx<float>*)h->h); }, &t[i])))
      return rc;
  }
  for (int i = 0; i < 2; ++i) {
    h->tune_pb = pbs[i];
    if ((rc = time_launches(h, reps, [&]() { return launch_reduce<float>(h, (const cx<float>*)h->J,
                                                                         (const cx<float>*)h->E, nullptr); },
                            &t[3 + i])))
      return rc;
  }
  best_ct = cts[t[0] <= t[1] ? (t[0] <= t[2] ? 0 : 2) : (t[1] <= t[2] ? 1 : 2)];
  best_pb = pbs[t[3] <= t[4] ? 0 : 1];
  h->tune_ct = best_ct;
  h->tune_pb = best_pb;
  // FFT plans of the two convolution kernels, timed inside the whole loss-gradient pass (their
  // speed depends on the kernels around them); scratch in and out: g0 as coefficients, the Adam
  // moment m (re-initialised by every reconstruction) as the gradient, loss_w as the loss record
  // (where the full tile does not fit, only plan 0 exists: its time stands for all four)
  const int nplans = full_tile_fits(h->M) ? 4 : 1;
  int best_plan = 0;
  for (int i = 0; i < nplans; ++i) {
    h->tune_fpp = i >> 1;
    h->tune_app = i & 1;
    if ((rc = time_launches(h, reps, [&]() {
           return run_iteration<float>(h, h->g0, h->m, h->loss_w, nullptr, nullptr, nullptr, nullptr, nullptr);
         }, &t[5 + i])))
      return rc;
    if (t[5 + i] < t[5 + best_plan]) best_plan = i;
  }
  for (int i = nplans; i < 4; ++i) t[5 + i] = t[5];
  h->tune_fpp = best_plan >> 1;
  h->tune_app = best_plan & 1;
  h->tuned = true;
  if (choice) choice[0] = best_ct, choice[1] = best_pb, choice[2] = h->tune_fpp, choice[3] = h->tune_app;
  if (ms)
    for (int i = 0; i < 9; ++i) ms[i] = t[i];
  return PDF_OK;
}

extern "C" int pdf_set_tiles(pdf_handle* h, int32_t ct, int32_t pb, int32_t fwd_pp, int32_t adj_pp) {
  if (!h || (ct != 1 && ct != 2 && ct != 4) || (pb != 4 && pb != 8) || (fwd_pp != 0 && fwd_pp != 1) ||
      (adj_pp != 0 && adj_pp != 1))
    return fail(h, PDF_EINVAL, "bad tile choice");
  for (int f = 0; f < h->F && h->F > 1; ++f) pdf_set_tiles(h->sub[f], ct, pb, fwd_pp, adj_pp);
  h->tune_ct = ct;
  h->tune_pb = pb;
  h->tune_fpp = fwd_pp;
  h->tune_app = adj_pp;
  h->tuned = true;
  return PDF_OK;
}

extern "C" int pdf_warm_start(pdf_handle* h, pdf_mlp* net, float s_in, float s_out, void* alpha_dev,
                              int32_t* chosen_dev, double* loss_dev) {
  if (!h || !net || !alpha_dev) return fail(h, PDF_EINVAL, "null argument");
  if (h->F > 1) return fail(h, PDF_EUNSUPPORTED, "the warm start covers single-frequency handles");
  if (!h->data_set) return fail(h, PDF_EINVAL, "pdf_set_data has not been called");
  if (h->prec != PDF_FP32) return fail(h, PDF_EUNSUPPORTED, "the warm start serves FP32 handles");
  int32_t n_in = 0, n_out = 0, bmax = 0;
  pdf_mlp_widths(net, &n_in, &n_out, &bmax);
  const int KK = h->K * h->K;
  if (n_in != 2 * h->Ni * h->Ns || n_out != 2 * h->Ni * KK)
    return fail(h, PDF_EINVAL, "network widths do not match 2 Ni Ns inputs and 2 Ni K^2 outputs");
  int rc;
  if ((rc = run_init<float>(h, alpha_dev))) return rc;
  if ((rc = run_loss<float>(h, alpha_dev, h->loss))) return rc;
  // the network's prediction into g0 (free after run_init), ordered between the two streams
  hipStream_t ns = pdf_mlp_stream(net);
  hipEvent_t ev;
  HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  rc = PDF_OK;
  if (hipEventRecord(ev, h->stream) != hipSuccess || hipStreamWaitEvent(ns, ev, 0) != hipSuccess)
    rc = fail(h, PDF_EHIP, "stream ordering failed");
  for (int b0 = 0; !rc && b0 < h->B; b0 += bmax) {
    const int nb = std::min(bmax, h->B - b0);
    if (pdf_mlp_forward(net, (const float*)h->esca + size_t(b0) * n_in, s_in, s_out, nb,
                        (float*)h->g0 + size_t(b0) * n_out))
      rc = fail(h, PDF_EHIP, std::string("network forward: ") + pdf_last_error(nullptr));
  }
  if (!rc && (hipEventRecord(ev, ns) != hipSuccess || hipStreamWaitEvent(h->stream, ev, 0) != hipSuccess))
    rc = fail(h, PDF_EHIP, "stream ordering failed");
  (void)hipEventDestroy(ev);
  if (rc) return rc;
  if ((rc = run_loss<float>(h, h->g0, h->loss_w))) return rc;
  const int len = h->Ni * KK;
  hipLaunchKernelGGL(k_pick_start<float>, dim3((len + 255) / 256, h->B), dim3(256), 0, h->stream,
                     (cx<float>*)alpha_dev, (const cx<float>*)h->g0, h->loss, h->loss_w, len, chosen_dev, loss_dev);
  return check_launch(h, "k_pick_start");
}

// ------------------------------------------------------------------ coefficient network

// Sizes of the network of a handle with hidden width H, its workspace
// (activations A1, A2, pre-activation gradients G1, G2, the gradient g at
// alpha_hat) and the launches of one forward pass or one step.
template <typename T>
struct FcNet {
  int R = 0, Q = 0, D = 0, H = 0, B = 0;
  size_t P = 0, off[3] = {0, 0, 0};
  T *A1 = nullptr, *A2 = nullptr, *G1 = nullptr, *G2 = nullptr;
  cx<T>* g = nullptr;
  T *X = nullptr, *G3 = nullptr, *Y = nullptr;   // real [Re | Im] rows (FP32 path): s_in alpha_0, s_out g, output
};

static size_t fc_params(int K, int H) {
  const size_t D = size_t(2) * K * K;
  return (D + 1) * H + size_t(H + 1) * H + size_t(H + 1) * D;
}

template <typename T>
static int fc_prepare(pdf_handle* h, int H, FcNet<T>* n) {
  if (H < 1 || H > 4096) return fail(h, PDF_EINVAL, "hidden width outside 1..4096");
  if (h->Ni > kFcMaxRows) return fail(h, PDF_EUNSUPPORTED, "the coefficient network takes at most 64 incidences");
  n->R = h->Ni;
  n->Q = h->K * h->K;
  n->D = 2 * n->Q;
  n->H = H;
  n->B = h->B;
  n->off[0] = 0;
  n->off[1] = size_t(n->D + 1) * H;
  n->off[2] = n->off[1] + size_t(H + 1) * H;
  n->P = fc_params(h->K, H);
  const size_t rows = size_t(h->B) * n->R;
  const size_t hid = rows * H * sizeof(T), gb = rows * n->Q * sizeof(cx<T>);
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t need = 4 * al(hid) + 4 * al(gb);
  if (h->fc_bytes < need) {
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (h->fc_ws) HIP_TRY(hipFree(h->fc_ws));
    h->fc_ws = nullptr;
    h->fc_bytes = 0;
    HIP_TRY(hipMalloc(&h->fc_ws, need));
    h->fc_bytes = need;
  }
  unsigned char* w = static_cast<unsigned char*>(h->fc_ws);
  n->A1 = reinterpret_cast<T*>(w);
  n->A2 = reinterpret_cast<T*>(w + al(hid));
  n->G1 = reinterpret_cast<T*>(w + 2 * al(hid));
  n->G2 = reinterpret_cast<T*>(w + 3 * al(hid));
  n->g = reinterpret_cast<cx<T>*>(w + 4 * al(hid));
  n->X = reinterpret_cast<T*>(w + 4 * al(hid) + al(gb));
  n->G3 = reinterpret_cast<T*>(w + 4 * al(hid) + 2 * al(gb));
  n->Y = reinterpret_cast<T*>(w + 4 * al(hid) + 3 * al(gb));
  return PDF_OK;
}

template <typename T>
static FcRows<T> fc_real(const T* p, int width) {
  FcRows<T> r;
  r.re = p;
  r.width = width;
  return r;
}

template <typename T>
static FcRows<T> fc_split(const cx<T>* p, int width, double scale) {
  FcRows<T> r;
  r.cxv = p;
  r.width = width;
  r.scale = T(scale);
  return r;
}

template <typename T, int RPW>
static void fc_launch(pdf_handle* h, const FcLayerArgs<T>& a, int kind) {
  const size_t lds = sizeof(T) * (size_t(kFcMaxRows) * kFcRed + size_t(kFcRed) * (kFcCols + 1));
  if (kind == 0) {
    set_lds(k_fc_fwd<T, RPW, false>, lds);
    hipLaunchKernelGGL((k_fc_fwd<T, RPW, false>), dim3((a.n_out + kFcCols - 1) / kFcCols, h->B), dim3(256), lds,
                       h->stream, a);
  } else if (kind == 1) {
    set_lds(k_fc_fwd<T, RPW, true>, lds);
    hipLaunchKernelGGL((k_fc_fwd<T, RPW, true>), dim3((a.n_out + kFcCols - 1) / kFcCols, h->B), dim3(256), lds,
                       h->stream, a);
  } else {
    set_lds(k_fc_bwd<T, RPW>, lds);
    hipLaunchKernelGGL((k_fc_bwd<T, RPW>), dim3((a.n_in + kFcCols - 1) / kFcCols, h->B), dim3(256), lds, h->stream,
                       a);
  }
}

template <int RT>
static void fc_launch_mfma(pdf_handle* h, const FcLayerArgs<float>& a, int kind) {
  const size_t lds = kFcMfmaLds;
  if (kind == 0) {
    set_lds(k_fc_fwd_mfma<RT, false>, lds);
    hipLaunchKernelGGL((k_fc_fwd_mfma<RT, false>), dim3((a.n_out + kFcCols - 1) / kFcCols * h->B), dim3(256), lds,
                       h->stream, a);
  } else if (kind == 1) {
    set_lds(k_fc_fwd_mfma<RT, true>, lds);
    hipLaunchKernelGGL((k_fc_fwd_mfma<RT, true>), dim3((a.n_out + kFcCols - 1) / kFcCols * h->B), dim3(256), lds,
                       h->stream, a);
  } else {
    set_lds(k_fc_bwd_mfma<RT>, lds);
    hipLaunchKernelGGL((k_fc_bwd_mfma<RT>), dim3((a.n_in + kFcCols - 1) / kFcCols * h->B), dim3(256), lds, h->stream,
                       a);
  }
}

// kind 0: hidden forward layer, 1: output layer, 2: hidden pre-activation gradient.
// FP32 runs on the matrix cores, FP64 on the vector units.
template <typename T>
static int fc_layer(pdf_handle* h, const FcLayerArgs<T>& a, int kind) {
  if constexpr (sizeof(T) == 4) {
    if (a.R <= 32) fc_launch_mfma<1>(h, a, kind);
    else fc_launch_mfma<2>(h, a, kind);
    return check_launch(h, kind == 2 ? "k_fc_bwd_mfma" : "k_fc_fwd_mfma");
  }
  const int rpw = (a.R + 3) / 4;
  if (rpw <= 1) fc_launch<T, 1>(h, a, kind);
  else if (rpw <= 2) fc_launch<T, 2>(h, a, kind);
  else if (rpw <= 4) fc_launch<T, 4>(h, a, kind);
  else if (rpw <= 8) fc_launch<T, 8>(h, a, kind);
  else fc_launch<T, 16>(h, a, kind);
  return check_launch(h, kind == 2 ? "k_fc_bwd" : "k_fc_fwd");
}

template <typename T>
static FcLayerArgs<T> fc_layer_args(const FcNet<T>& n, int l, const T* theta) {
  FcLayerArgs<T> a{};
  a.theta = theta + n.off[l];
  a.theta_stride = n.P;
  a.R = n.R;
  a.n_in = l == 0 ? n.D : n.H;
  a.n_out = l == 2 ? n.D : n.H;
  return a;
}

// [Re | Im] real rows of complex rows (FP32 path).
template <typename T>
static int fc_split_rows(pdf_handle* h, const FcNet<T>& n, const cx<T>* z, double scale, T* out) {
  const size_t cnt = size_t(n.B) * n.R * n.Q;
  hipLaunchKernelGGL(k_fc_split<T>, dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, h->stream, z, T(scale), out,
                     n.Q, cnt);
  return check_launch(h, "k_fc_split");
}

// alpha_hat = alpha_0 + s_out f_theta(s_in alpha_0); activations kept in the workspace.  The
// FP32 path takes the network's real rows from n.X and joins the output rows n.Y into alpha_hat.
template <typename T>
static int fc_forward(pdf_handle* h, const FcNet<T>& n, const cx<T>* alpha0, const T* theta, cx<T>* alpha_hat,
                      double s_in, double s_out) {
  int rc;
  constexpr bool F32 = sizeof(T) == 4;
  FcLayerArgs<T> a = fc_layer_args(n, 0, theta);
  if (F32) {
    if ((rc = fc_split_rows<T>(h, n, alpha0, s_in, n.X))) return rc;
    a.in = fc_real<T>(n.X, n.D);
    a.in_stride = size_t(n.R) * n.D;
  } else {
    a.in = fc_split(alpha0, n.D, s_in);
    a.in_stride = size_t(n.R) * n.Q;
  }
  a.act = n.A1;
  if ((rc = fc_layer(h, a, 0))) return rc;
  a = fc_layer_args(n, 1, theta);
  a.in = fc_real<T>(n.A1, n.H);
  a.in_stride = size_t(n.R) * n.H;
  a.act = n.A2;
  if ((rc = fc_layer(h, a, 0))) return rc;
  a = fc_layer_args(n, 2, theta);
  a.in = fc_real<T>(n.A2, n.H);
  a.in_stride = size_t(n.R) * n.H;
  a.alpha0 = alpha0;
  a.alpha_hat = alpha_hat;
  a.out_scale = T(s_out);
  a.act = n.Y;
  if ((rc = fc_layer(h, a, 1))) return rc;
  if (!F32) return PDF_OK;
  const size_t cnt = size_t(n.B) * n.R * n.Q;
  hipLaunchKernelGGL(k_fc_join<T>, dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, h->stream, alpha0,
                     (const T*)n.Y, T(s_out), alpha_hat, n.Q, cnt);
  return check_launch(h, "k_fc_join");
}

template <typename T>
static int fc_step(pdf_handle* h, int H, double s_in, double s_out, const cx<T>* alpha0, T* theta, T* m, T* v,
                   int t, cx<T>* alpha_hat, double* loss) {
  FcNet<T> n;
  int rc;
  if ((rc = fc_prepare<T>(h, H, &n))) return rc;
  if ((rc = fc_forward<T>(h, n, alpha0, theta, alpha_hat, s_in, s_out))) return rc;
  if ((rc = run_iteration<T>(h, alpha_hat, n.g, loss, nullptr, nullptr, nullptr, nullptr, nullptr))) return rc;
  // pre-activation gradients with the weights before the update; dL/dY = s_out [Re g | Im g]
  constexpr bool F32 = sizeof(T) == 4;
  FcLayerArgs<T> a = fc_layer_args(n, 2, theta);
  if (F32) {
    if ((rc = fc_split_rows<T>(h, n, n.g, s_out, n.G3))) return rc;
    a.in = fc_real<T>(n.G3, n.D);
    a.in_stride = size_t(n.R) * n.D;
  } else {
    a.in = fc_split<T>(n.g, n.D, s_out);
    a.in_stride = size_t(n.R) * n.Q;
  }
  a.a_prev = n.A2;
  a.gprev = n.G2;
  if ((rc = fc_layer(h, a, 2))) return rc;
  a = fc_layer_args(n, 1, theta);
  a.in = fc_real<T>(n.G2, n.H);
  a.in_stride = size_t(n.R) * n.H;
  a.a_prev = n.A1;
  a.gprev = n.G1;
  if ((rc = fc_layer(h, a, 2))) return rc;
  FcAdamArgs<T> d{};
  d.in[0] = F32 ? fc_real<T>(n.X, n.D) : fc_split(alpha0, n.D, s_in);
  d.in_stride[0] = size_t(n.R) * (F32 ? n.D : n.Q);
  d.in[1] = fc_real<T>(n.A1, n.H);
  d.in[2] = fc_real<T>(n.A2, n.H);
  d.in_stride[1] = d.in_stride[2] = size_t(n.R) * n.H;
  d.g[0] = fc_real<T>(n.G1, n.H);
  d.g[1] = fc_real<T>(n.G2, n.H);
  d.g_stride[0] = d.g_stride[1] = size_t(n.R) * n.H;
  d.g[2] = F32 ? fc_real<T>(n.G3, n.D) : fc_split<T>(n.g, n.D, s_out);
  d.g_stride[2] = size_t(n.R) * (F32 ? n.D : n.Q);
  // two columns per lane where every width and block offset is even (H even; D = 2 K^2 always is)
  const bool v2 = F32 && n.H % 2 == 0 && n.P % 2 == 0;
  const int rows_t = v2 ? FcAdamTile<2>::ROWS : FcAdamTile<1>::ROWS;
  const int cols_t = v2 ? FcAdamTile<2>::COLS : FcAdamTile<1>::COLS;
  d.tile_start[0] = 0;
  for (int l = 0; l < 3; ++l) {
    d.n_in[l] = l == 0 ? n.D : n.H;
    d.n_out[l] = l == 2 ? n.D : n.H;
    d.off[l] = n.off[l];
    const int tiles = ((d.n_in[l] + 1 + rows_t - 1) / rows_t) * ((d.n_out[l] + cols_t - 1) / cols_t);
    d.tile_start[l + 1] = d.tile_start[l] + tiles;
  }
  if (int64_t(d.tile_start[3]) * h->B > INT32_MAX) return fail(h, PDF_EINVAL, "k_fc_adam: grid too large");
  d.R = n.R;
  d.xcd_order = h->B % 8 == 0;
  d.theta = theta;
  d.m = m;
  d.v = v;
  d.theta_stride = n.P;
  d.b1 = h->prm.adam_b1;
  d.b2 = h->prm.adam_b2;
  d.eps = h->prm.adam_eps;
  d.lr1 = h->prm.lr / (1.0 - std::pow(h->prm.adam_b1, double(t)));
  d.ic2 = 1.0 / (1.0 - std::pow(h->prm.adam_b2, double(t)));
  if constexpr (F32) {
    if (v2) {
      hipLaunchKernelGGL((k_fc_adam<T, 2>), dim3(d.tile_start[3] * h->B), dim3(256), 0, h->stream, d);
      return check_launch(h, "k_fc_adam");
    }
  }
  hipLaunchKernelGGL((k_fc_adam<T, 1>), dim3(d.tile_start[3] * h->B), dim3(256), 0, h->stream, d);
  return check_launch(h, "k_fc_adam");
}

extern "C" int pdf_fcnn_size(const pdf_handle* h, int32_t hidden, int64_t* n_params) {
  if (!h || !n_params) return fail(nullptr, PDF_EINVAL, "pdf_fcnn_size: null argument");
  if (hidden < 1 || hidden > 4096) return fail(nullptr, PDF_EINVAL, "pdf_fcnn_size: hidden width outside 1..4096");
  *n_params = int64_t(fc_params(h->K, hidden));
  return PDF_OK;
}

static int fc_check_scales(pdf_handle* h, double s_in, double s_out) {
  if (!std::isfinite(s_in) || !std::isfinite(s_out)) return fail(h, PDF_EINVAL, "s_in and s_out must be finite");
  return PDF_OK;
}

extern "C" int pdf_fcnn_forward(pdf_handle* h, int32_t hidden, double s_in, double s_out, const void* alpha0_dev,
                                const void* theta_dev, void* alpha_hat_dev) {
  if (!h || !alpha0_dev || !theta_dev || !alpha_hat_dev) return fail(h, PDF_EINVAL, "null argument");
  if (h->F > 1) return fail(h, PDF_EUNSUPPORTED, "the coefficient network covers single-frequency handles");
  if (alpha_hat_dev == alpha0_dev) return fail(h, PDF_EINVAL, "alpha_hat must not alias alpha_0");
  int rc;
  if ((rc = fc_check_scales(h, s_in, s_out))) return rc;
  if (h->prec == PDF_FP32) {
    FcNet<float> n;
    if ((rc = fc_prepare<float>(h, hidden, &n))) return rc;
    return fc_forward<float>(h, n, (const cx<float>*)alpha0_dev, (const float*)theta_dev, (cx<float>*)alpha_hat_dev,
                             s_in, s_out);
  }
  FcNet<double> n;
  if ((rc = fc_prepare<double>(h, hidden, &n))) return rc;
  return fc_forward<double>(h, n, (const cx<double>*)alpha0_dev, (const double*)theta_dev,
                            (cx<double>*)alpha_hat_dev, s_in, s_out);
}

extern "C" int pdf_fcnn_step(pdf_handle* h, int32_t hidden, double s_in, double s_out, const void* alpha0_dev,
                             void* theta_dev, void* m_dev, void* v_dev, int32_t t, void* alpha_hat_dev,
                             double* loss_dev) {
  if (!h || !alpha0_dev || !theta_dev || !m_dev || !v_dev || !alpha_hat_dev)
    return fail(h, PDF_EINVAL, "null argument");
  if (h->F > 1) return fail(h, PDF_EUNSUPPORTED, "the coefficient network covers single-frequency handles");
  if (alpha_hat_dev == alpha0_dev) return fail(h, PDF_EINVAL, "alpha_hat must not alias alpha_0");
  if (t < 1) return fail(h, PDF_EINVAL, "the step number t counts from 1");
  if (!h->data_set) return fail(h, PDF_EINVAL, "pdf_set_data has not been called");
  if (int rc = fc_check_scales(h, s_in, s_out)) return rc;
  return h->prec == PDF_FP32
             ? fc_step<float>(h, hidden, s_in, s_out, (const cx<float>*)alpha0_dev, (float*)theta_dev,
                              (float*)m_dev, (float*)v_dev, t, (cx<float>*)alpha_hat_dev, loss_dev)
             : fc_step<double>(h, hidden, s_in, s_out, (const cx<double>*)alpha0_dev, (double*)theta_dev,
                               (double*)m_dev, (double*)v_dev, t, (cx<double>*)alpha_hat_dev, loss_dev);
}

template <typename T, int M>
static int launch_analyze_m(pdf_handle* h, int n, const void* J, void* alpha) {
  using C = ConvCfg<T, M>;
  if constexpr (C::LDS_BYTES <= 160 * 1024) {
    auto k = k_analyze<T, M>;
    set_lds(k, C::LDS_BYTES);
    hipLaunchKernelGGL(k, dim3(unsigned(n) * h->Ni), dim3(C::NT), C::LDS_BYTES, h->stream, (const cx<T>*)J,
                       (const cx<T>*)h->tw, (cx<T>*)alpha, h->K);
    return check_launch(h, "k_analyze");
  } else {
    return fail(h, PDF_EUNSUPPORTED, "grid too large for the LDS-resident transform");
  }
}

// alpha = F_T(J) for big grids: chunks of at most B sets through S.
template <typename T, int M>
static int launch_analyze_big_m(pdf_handle* h, int n, const void* J, void* alpha) {
  AdjArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  a.tw = (const cx<T>*)h->tw;
  a.Ni = h->Ni;
  a.K = h->K;
  const size_t per = size_t(h->Ni) * h->N, kk = size_t(h->Ni) * h->K * h->K;
  for (int c0 = 0; c0 < n; c0 += h->B) {
    const int cn = std::min(h->B, n - c0);
    a.galpha = (cx<T>*)alpha + size_t(c0) * kk;
    int rc = launch_adj_tail_big_m<T, M>(h, a, cn * h->Ni, (const cx<T>*)J + size_t(c0) * per, T(1) / T(h->N));
    if (rc) return rc;
  }
  return PDF_OK;
}

template <typename T>
static int launch_analyze(pdf_handle* h, int n, const void* J, void* alpha) {
  if (h->big) {
    switch (h->M) {
      case 128: return launch_analyze_big_m<T, 128>(h, n, J, alpha);
      case 256: return launch_analyze_big_m<T, 256>(h, n, J, alpha);
      case 96:
        if constexpr (sizeof(T) == 8) return launch_analyze_big_m<T, 96>(h, n, J, alpha);
        break;
    }
    return fail(h, PDF_EUNSUPPORTED, "unsupported M");
  }
  switch (h->M) {
    case 8: return launch_analyze_m<T, 8>(h, n, J, alpha);
    case 16: return launch_analyze_m<T, 16>(h, n, J, alpha);
    case 32: return launch_analyze_m<T, 32>(h, n, J, alpha);
    case 48: return launch_analyze_m<T, 48>(h, n, J, alpha);
    case 64: return launch_analyze_m<T, 64>(h, n, J, alpha);
    case 96: return launch_analyze_m<T, 96>(h, n, J, alpha);
  }
  return fail(h, PDF_EUNSUPPORTED, "unsupported M");
}

extern "C" int pdf_analyze(pdf_handle* h, int32_t n, const void* J_dev, void* alpha_dev) {
  if (!h || !J_dev || !alpha_dev) return fail(h, PDF_EINVAL, "null argument");
  if (h->F > 1) return fail(h, PDF_EUNSUPPORTED, "the analysis is per frequency: apply it to one frequency");
  if (n < 1) return fail(h, PDF_EINVAL, "n must be >= 1");
  return h->prec == PDF_FP32 ? launch_analyze<float>(h, n, J_dev, alpha_dev)
                             : launch_analyze<double>(h, n, J_dev, alpha_dev);
}

extern "C" int pdf_image(pdf_handle* h, const void* alpha_dev, void* chi_dev, void* chi_cco_dev,
                         const void* eps_true_dev, double* err_dev) {
  if (!h || !alpha_dev) return fail(h, PDF_EINVAL, "null argument");
  if (err_dev && !eps_true_dev) return fail(h, PDF_EINVAL, "err_dev needs eps_true_dev");
  return h->prec == PDF_FP32 ? run_image<float>(h, alpha_dev, chi_dev, chi_cco_dev, eps_true_dev, err_dev)
                             : run_image<double>(h, alpha_dev, chi_dev, chi_cco_dev, eps_true_dev, err_dev);
}

// One handle's part of a reconstruction: start value, counters, error checks,
// n_check captured iterations, final image.  Handles of either precision
// share the interface, so several can be advanced together.
struct Recon {
  virtual ~Recon() = default;
  virtual int prepare(int start_given) = 0;        // start value and counters; first error check
  virtual int check() = 0;                         // error check after a chunk (updates nf)
  virtual int iterate(int k) = 0;                  // k iterations on the handle's stream (capturable)
  virtual int finish() = 0;                        // final image, synchronise
  pdf_handle* h = nullptr;
  bool has_target = false;
  int nf = 0;                                      // instances that reached their target
  bool active() const { return nf < h->B; }
};

template <typename T>
struct ReconT : Recon {
  void* alpha;
  const void* eps_true;
  const double* target;
  int *reached, *best_iter;
  double* best_err;
  void* cco_out;
  std::vector<int> fz;
  ReconT(pdf_handle* hh, void* a, const void* et, const double* tg, int* re, double* be, int* bi, void* co)
      : alpha(a), eps_true(et), target(tg), reached(re), best_iter(bi), best_err(be), cco_out(co) {
    h = hh;
    has_target = tg != nullptr;
    fz.resize(hh->B);
  }
  int prepare(int start_given) override {
    int rc;
    const size_t KK = size_t(h->K) * h->K;
    const size_t nre = 2 * size_t(h->B) * h->Ni * KK;
    if (!start_given && (rc = run_init<T>(h, alpha))) return rc;
    const int tb = 256;
    const dim3 gb((h->B + tb - 1) / tb);
    hipLaunchKernelGGL(k_fill_zero<T>, dim3((nre + tb - 1) / tb), dim3(tb), 0, h->stream, (T*)h->m, nre);
    hipLaunchKernelGGL(k_fill_zero<T>, dim3((nre + tb - 1) / tb), dim3(tb), 0, h->stream, (T*)h->v, nre);
    hipLaunchKernelGGL(k_fill_int, gb, dim3(tb), 0, h->stream, h->tstep, 0, h->B);
    hipLaunchKernelGGL(k_fill_int, gb, dim3(tb), 0, h->stream, h->frozen, 0, h->B);
    if (reached) hipLaunchKernelGGL(k_fill_int, gb, dim3(tb), 0, h->stream, reached, -1, h->B);
    if (best_iter) hipLaunchKernelGGL(k_fill_int, gb, dim3(tb), 0, h->stream, best_iter, -1, h->B);
    if (best_err) hipLaunchKernelGGL(k_fill_double, gb, dim3(tb), 0, h->stream, best_err, HUGE_VAL, h->B);
    if ((rc = check_launch(h, "fill"))) return rc;
    nf = 0;
    return eps_true ? check() : PDF_OK;
  }
  int check() override {
    if (!eps_true) return PDF_OK;
    const int tb = 256;
    const dim3 gb((h->B + tb - 1) / tb);
    int r = run_image<T>(h, alpha, nullptr, nullptr, eps_true, h->err);
    if (r) return r;
    hipLaunchKernelGGL(k_track_error, gb, dim3(tb), 0, h->stream, h->err, target, h->frozen, reached, best_err,
                       best_iter, h->tstep, h->B);
    if ((r = check_launch(h, "k_track_error"))) return r;
    nf = 0;
    if (target) {
      HIP_TRY(hipMemcpyAsync(fz.data(), h->frozen, sizeof(int) * h->B, hipMemcpyDeviceToHost, h->stream));
      HIP_TRY(hipStreamSynchronize(h->stream));
      for (int x : fz) nf += x;
    }
    return PDF_OK;
  }
  int iterate(int k) override {
    for (int s = 0; s < k; ++s)
      if (int rc = run_iteration<T>(h, alpha, nullptr, h->loss, alpha, h->m, h->v, h->tstep, h->frozen)) return rc;
    return PDF_OK;
  }
  int finish() override {
    int rc;
    if (cco_out && (rc = run_image<T>(h, alpha, nullptr, cco_out, nullptr, nullptr))) return rc;
    HIP_TRY(hipStreamSynchronize(h->stream));
    return PDF_OK;
  }
};

// A unit advances one handle, or a shape class of handles by grouped launches.
struct Unit {
  std::vector<Recon*> rs;
  std::unique_ptr<Group> grp;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<hipEvent_t> evs;  // one per member: joins and forks of the members' streams
  ~Unit() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
  }
  pdf_handle* lead() const { return rs[0]->h; }
  bool active() const {
    for (Recon* r : rs)
      if (r->active()) return true;
    return false;
  }
  int iterate(int k) { return grp ? group_iterate(grp.get(), k) : rs[0]->iterate(k); }
  // the lead stream waits for every member's stream (before), or every member for the lead (after)
  int join(bool before) {
    pdf_handle* h = lead();
    if (rs.size() < 2) return PDF_OK;
    if (evs.empty()) {
      evs.resize(rs.size(), nullptr);
      for (auto& e : evs) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    if (before) {
      for (size_t i = 1; i < rs.size(); ++i) {
        HIP_TRY(hipEventRecord(evs[i], rs[i]->h->stream));
        HIP_TRY(hipStreamWaitEvent(h->stream, evs[i], 0));
      }
    } else {
      HIP_TRY(hipEventRecord(evs[0], h->stream));
      for (size_t i = 1; i < rs.size(); ++i) HIP_TRY(hipStreamWaitEvent(rs[i]->h->stream, evs[0], 0));
    }
    return PDF_OK;
  }
};

// Captures k iterations of a unit on its lead stream into a new graph.
static int capture_unit(Unit& u, int k, hipGraph_t* g) {
  pdf_handle* h = u.lead();
  *g = nullptr;
  HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  const int crc = u.iterate(k);
  hipError_t ce = hipStreamEndCapture(h->stream, g);
  if (crc) {
    if (*g) (void)hipGraphDestroy(*g);
    *g = nullptr;
    return crc;
  }
  if (ce != hipSuccess) return fail(h, PDF_EHIP, std::string("capture: ") + hipGetErrorString(ce));
  return PDF_OK;
}

// Advances every unit together.  Each unit's n_check steps are captured once
// into a graph of its own and launched on its lead handle's stream, so
// different units overlap on the hardware queues while a unit's grouped
// launches fill the GPU with all of its handles' work; checks and early stop
// are per handle.
static int reconstruct_all(std::vector<std::unique_ptr<Unit>>& units, int n_iter, int n_check, int start_given,
                           pdf_report* rep) {
  auto t0 = std::chrono::steady_clock::now();
  int rc = PDF_OK;
  for (auto& u : units)
    for (Recon* r : u->rs)
      if ((rc = r->prepare(start_given))) return rc;
  if (n_check < 1 || n_check > n_iter) n_check = n_iter > 0 ? n_iter : 1;
  int done = 0;
  while (!rc && done < n_iter) {
    bool any = false;
    const int chunk = (n_iter - done < n_check) ? n_iter - done : n_check;
    for (auto& up : units) {
      Unit& u = *up;
      if (rc || !u.active()) continue;
      any = true;
      if ((rc = u.join(true))) break;
      if (chunk == n_check) {
        if (!u.exec) {
          if ((rc = capture_unit(u, n_check, &u.graph))) break;
          hipError_t ie = hipGraphInstantiate(&u.exec, u.graph, nullptr, nullptr, 0);
          if (ie != hipSuccess) {
            rc = fail(u.lead(), PDF_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
            break;
          }
        }
        hipError_t le = hipGraphLaunch(u.exec, u.lead()->stream);
        if (le != hipSuccess) rc = fail(u.lead(), PDF_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(le));
      } else {
        rc = u.iterate(chunk);
      }
      if (!rc) rc = u.join(false);
    }
    if (!any) break;
    done += chunk;
    for (auto& u : units)
      for (Recon* r : u->rs)
        if (!rc && r->active()) rc = r->check();
  }
  if (rc) return rc;
  int reached = 0;
  bool any_target = false;
  for (auto& u : units)
    for (Recon* r : u->rs) {
      if ((rc = r->finish())) return rc;
      reached += r->nf;
      any_target = any_target || r->has_target;
    }
  if (rep) {
    rep->iters_run = done;
    rep->n_reached = any_target ? reached : 0;
    rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return PDF_OK;
}

static Recon* make_recon(pdf_handle* h, void* alpha, const void* eps_true, const double* target, int* reached,
                         double* best_err, int* best_iter, void* cco_out) {
  if (h->prec == PDF_FP32) return new ReconT<float>(h, alpha, eps_true, target, reached, best_err, best_iter, cco_out);
  return new ReconT<double>(h, alpha, eps_true, target, reached, best_err, best_iter, cco_out);
}

static int check_recon_args(pdf_handle* h, void* alpha_dev, int n_iter, const void* eps_true_dev,
                            const double* target_err_dev, const double* best_err_dev) {
  if (!h || !alpha_dev) return fail(h, PDF_EINVAL, "null argument");
  if (n_iter < 0) return fail(h, PDF_EINVAL, "n_iter < 0");
  if (!h->data_set) return fail(h, PDF_EINVAL, "pdf_set_data has not been called");
  if ((target_err_dev || best_err_dev) && !eps_true_dev)
    return fail(h, PDF_EINVAL, "error tracking needs eps_true_dev");
  return PDF_OK;
}

extern "C" int pdf_reconstruct(pdf_handle* h, int32_t n_iter, int32_t n_check, int32_t start_given,
                               void* alpha_dev, const void* eps_true_dev, const double* target_err_dev,
                               int32_t* reached_iter_dev, double* best_err_dev, int32_t* best_iter_dev,
                               void* chi_cco_dev, pdf_report* rep) {
  if (int rc = check_recon_args(h, alpha_dev, n_iter, eps_true_dev, target_err_dev, best_err_dev)) return rc;
  std::unique_ptr<Recon> r(make_recon(h, alpha_dev, eps_true_dev, target_err_dev, reached_iter_dev, best_err_dev,
                                      best_iter_dev, chi_cco_dev));
  std::vector<std::unique_ptr<Unit>> units;
  units.emplace_back(new Unit());
  units[0]->rs.push_back(r.get());
  return reconstruct_all(units, n_iter, n_check, start_given, rep);
}

extern "C" int pdf_reconstruct_multi(int32_t n, pdf_handle* const* hs, int32_t n_iter, int32_t n_check,
                                     int32_t start_given, void* const* alpha_dev, const void* const* eps_true_dev,
                                     const double* const* target_err_dev, int32_t* const* reached_iter_dev,
                                     double* const* best_err_dev, int32_t* const* best_iter_dev,
                                     void* const* chi_cco_dev, pdf_report* rep) {
  if (n < 1 || !hs || !alpha_dev) return fail(nullptr, PDF_EINVAL, "pdf_reconstruct_multi: null argument");
  std::vector<std::unique_ptr<Recon>> own;
  std::vector<Recon*> rs;
  for (int i = 0; i < n; ++i) {
    const void* et = eps_true_dev ? eps_true_dev[i] : nullptr;
    const double* tg = target_err_dev ? target_err_dev[i] : nullptr;
    double* be = best_err_dev ? best_err_dev[i] : nullptr;
    if (int rc = check_recon_args(hs[i], alpha_dev[i], n_iter, et, tg, be)) return rc;
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(hs[i], PDF_EINVAL, "a handle appears twice");
    own.emplace_back(make_recon(hs[i], alpha_dev[i], et, tg, reached_iter_dev ? reached_iter_dev[i] : nullptr, be,
                                best_iter_dev ? best_iter_dev[i] : nullptr, chi_cco_dev ? chi_cco_dev[i] : nullptr));
    rs.push_back(own.back().get());
  }
  // shape classes of FP32 handles: one tile choice each (tuned on the member with the largest batch)
  std::map<std::array<int, 5>, std::vector<int>> classes;
  std::vector<std::unique_ptr<Unit>> units;
  for (int i = 0; i < n; ++i) {
    pdf_handle* h = hs[i];
    if (h->prec == PDF_FP32 && h->N % 32 == 0 && !h->big && h->F == 1 && !h->prm.cco_in_loss)
      classes[{h->M, (h->Ns + 15) / 16, (h->Ni + 31) / 32, (h->Ni + 15) / 16, compact_mode(h)}].push_back(i);
    else {
      units.emplace_back(new Unit());
      units.back()->rs.push_back(rs[i]);
    }
  }
  for (auto& kv : classes) {
    const std::vector<int>& idx = kv.second;
    int best = idx[0];
    for (int i : idx)
      if (hs[i]->B > hs[best]->B) best = i;
    if (!hs[best]->tuned)
      if (int rc = pdf_autotune(hs[best], 5, nullptr, nullptr)) return rc;
    for (int i : idx)
      pdf_set_tiles(hs[i], hs[best]->tune_ct, hs[best]->tune_pb, hs[best]->tune_fpp, hs[best]->tune_app);
    units.emplace_back(new Unit());
    Unit& u = *units.back();
    for (int i : idx) u.rs.push_back(rs[i]);
    if (idx.size() >= 2) {
      std::vector<pdf_handle*> gh;
      std::vector<void*> ga;
      for (int i : idx) {
        gh.push_back(hs[i]);
        ga.push_back(alpha_dev[i]);
      }
      u.grp.reset(new Group());
      if (int rc = group_build(u.grp.get(), gh, ga)) return rc;
    }
  }
  return reconstruct_all(units, n_iter, n_check, start_given, rep);
}

static int step_multi_impl(int32_t n, pdf_handle* const* hs, void* const* alpha_dev, void* const* m_dev,
                           void* const* v_dev, int32_t* const* t_dev, double* const* loss_dev);

extern "C" int pdf_step_multi(int32_t n, pdf_handle* const* hs, void* const* alpha_dev, void* const* m_dev,
                              void* const* v_dev, int32_t* const* t_dev, double* const* loss_dev) {
  g_last_error = "no error";
  for (int i = 0; hs && i < n; ++i)
    if (hs[i]) hs[i]->err_msg.clear();
  const int rc = step_multi_impl(n, hs, alpha_dev, m_dev, v_dev, t_dev, loss_dev);
  // the message of a failure goes to pdf_last_error(NULL) whichever handle it came from
  for (int i = 0; rc && hs && i < n; ++i)
    if (hs[i] && !hs[i]->err_msg.empty()) {
      g_last_error = "handle " + std::to_string(i) + ": " + hs[i]->err_msg;
      break;
    }
  return rc;
}

static int step_multi_impl(int32_t n, pdf_handle* const* hs, void* const* alpha_dev, void* const* m_dev,
                           void* const* v_dev, int32_t* const* t_dev, double* const* loss_dev) {
  if (n < 1 || !hs || !alpha_dev || !m_dev || !v_dev || !t_dev) return fail(nullptr, PDF_EINVAL, "pdf_step_multi: null argument");
  for (int i = 0; i < n; ++i) {
    if (!hs[i] || !alpha_dev[i] || !m_dev[i] || !v_dev[i] || !t_dev[i])
      return fail(nullptr, PDF_EINVAL, "pdf_step_multi: null entry " + std::to_string(i));
    if (!hs[i]->data_set) return fail(hs[i], PDF_EINVAL, "pdf_set_data has not been called");
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(hs[i], PDF_EINVAL, "a handle appears twice");
  }
  // shape classes of FP32 handles as in pdf_reconstruct_multi; the class's first member's tile
  // choice serves all (every choice computes the same values)
  std::map<std::array<int, 5>, std::vector<int>> classes;
  std::vector<int> single;
  for (int i = 0; i < n; ++i) {
    pdf_handle* h = hs[i];
    if (h->prec == PDF_FP32 && h->N % 32 == 0 && !h->big && h->F == 1 && !h->prm.cco_in_loss)
      classes[{h->M, (h->Ns + 15) / 16, (h->Ni + 31) / 32, (h->Ni + 15) / 16, compact_mode(h)}].push_back(i);
    else
      single.push_back(i);
  }
  auto loss_of = [&](int i) { return loss_dev ? loss_dev[i] : nullptr; };
  for (auto& kv : classes)
    if (kv.second.size() == 1) single.push_back(kv.second[0]);
  for (int i : single)
    if (int rc = pdf_step(hs[i], alpha_dev[i], m_dev[i], v_dev[i], t_dev[i], loss_of(i))) return rc;
  for (auto& kv : classes) {
    const std::vector<int>& idx = kv.second;
    if (idx.size() < 2) continue;
    std::vector<pdf_handle*> gh;
    std::vector<void*> ga;
    StepBufs sb;
    for (int i : idx) {
      gh.push_back(hs[i]);
      ga.push_back(alpha_dev[i]);
      sb.m.push_back(m_dev[i]);
      sb.v.push_back(v_dev[i]);
      sb.t.push_back(t_dev[i]);
      sb.loss.push_back(loss_of(i));
    }
    pdf_handle* h = gh[0];
    Group g;
    if (int rc = group_build(&g, gh, ga, &sb)) return rc;
    // the lead stream waits for every member's stream, runs the grouped step, and every member's
    // stream waits for it
    std::vector<hipEvent_t> ev(gh.size(), nullptr);
    for (auto& e : ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (size_t k = 1; k < gh.size(); ++k) {
      HIP_TRY(hipEventRecord(ev[k], gh[k]->stream));
      HIP_TRY(hipStreamWaitEvent(h->stream, ev[k], 0));
    }
    const int rc = group_iterate(&g, 1);
    HIP_TRY(hipEventRecord(ev[0], h->stream));
    for (size_t k = 1; k < gh.size(); ++k) HIP_TRY(hipStreamWaitEvent(gh[k]->stream, ev[0], 0));
    // the argument table is freed when g leaves this scope: wait for the launches that read it
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (rc) return rc;
  }
  return PDF_OK;
}

extern "C" const char* pdf_last_error(const pdf_handle* h) {
  return h ? h->err_msg.c_str() : g_last_error.c_str();
}
