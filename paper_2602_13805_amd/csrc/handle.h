// Internal state of a pdf_handle and shared host helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/pdf.h"

struct pdf_handle {
  int prec = PDF_FP32;
  int M = 0, N = 0, P = 0, K = 0, Ni = 0, Ns = 0, B = 0;
  int tile = 256, ntiles = 0;
  pdf_params prm{};
  hipStream_t stream = nullptr;
  int device = -1;                // device current at pdf_setup
  void* scratch_dev = nullptr;    // that device's copy of the library's static scratch
  std::string scratch_err;        // why scratch_dev is null, if it is
  // operator tables (handle precision)
  void* ghat = nullptr;   // [P][P] spectrum / P^2
  void* tw = nullptr;     // [P + M] exp(-2 pi i k / P), then the half-shift values hs[m]
  void* gs = nullptr;     // [Ns][N]
  void* gsT = nullptr;    // [N][Ns] (transposed copy for the MFMA receiver GEMM)
  float* gsA = nullptr;   // FP32: [N][ceil(Ns/16)][64] A operands of that GEMM in lane order
  void* einc = nullptr;   // [Ni][N]
  double* Ss = nullptr;   // device scalar ||E_inc||^2
  double* Sd = nullptr;   // device [B] ||E_sca||^2
  void* esca = nullptr;   // [B][Ni][Ns]
  bool data_set = false;
  // per-iteration scratch
  void* J = nullptr;      // [B][Ni][N]
  void* E = nullptr;      // [B][Ni][N]
  void* h = nullptr;      // [B][Ni][N]
  void* R = nullptr;      // [B][N]
  void* den = nullptr;    // [B][N] real
  void* chi = nullptr;    // [B][N]
  void* gR = nullptr;     // [B][N]
  void* Dpart = nullptr;  // [B][ntiles][Ni][Ns]
  void* dres = nullptr;   // [B][Ni][Ns]
  double* lsp = nullptr;  // [B][ntiles]
  // start-value and reconstruction scratch
  void* R0 = nullptr;     // [B][N]
  void* g0 = nullptr;     // [B][Ni][K][K]
  double* gnorm = nullptr;   // [B]
  double* err = nullptr;     // [B]
  int* frozen = nullptr;     // [B]
  int* tstep = nullptr;      // [B]
  double* adam_c = nullptr;  // [B][2] Adam bias corrections of the current step
  void* m = nullptr;         // [B][Ni][K][K][2] real
  void* v = nullptr;
  double* loss = nullptr;    // [B][8]
  double* loss_w = nullptr;  // [B][8] second loss record (start selection)
  // grids whose padded half tile exceeds one CU's LDS run the convolution in
  // passes through S; GJ holds g_J between the adjoint's passes; big_ws the
  // CCO filter coefficients [B][4][N] and error parts [B][ceil(N/256)][2]
  bool big = false;
  void* S = nullptr;        // [B][Ni][M][2M]
  void* GJ = nullptr;       // [B][Ni][N]
  void* big_ws = nullptr;
  // the loss on the CCO image (cco_in_loss): filter workspace [B][kCclArrays][N],
  // chi_c and R_c [B][N], per-workgroup state sums [B][ceil(N / 256)]
  void* ccl_ws = nullptr;
  void* chic = nullptr;
  void* Rc = nullptr;
  double* ccl_part = nullptr;
  double* reg_part = nullptr;  // big grids: per-workgroup sums of the regulariser pass [B][ceil(N / 256)][6]
  // several frequencies: F > 1 makes this handle the container of one handle
  // per frequency (batch 1 each), joined through the shared contrast; its own
  // per-pixel buffers (R, den, chi, gR, lsp) hold the joint values
  int F = 1;
  pdf_handle* sub[8] = {};
  double* mf_wsum = nullptr;   // a frequency handle: where its pixel reduction writes weighted sums (or null)
  double mf_w = 1.0;           // and their weight 1 / ||E_inc||^2
  double ss_host = 0.0;        // ||E_inc||^2 on the host
  double* wsum = nullptr;      // container: [F][N][4] weighted pixel sums
  double* one = nullptr;       // container: device 1.0 (the joint state loss is weighted already)
  double* dn = nullptr;        // container: [F] ||G_S,f J_f - E_sca,f||^2
  double* gn = nullptr;        // container: [F] ||g_f||^2 of the start value
  double* sdf = nullptr;       // container: [F] ||E_sca,f||^2
  double* mf_dp = nullptr;     // container: [F][ceil(Ni Ns / 16)] parts of the start's ||G_S,f J_g||^2
  // coefficient-network workspace (activations and gradients of one step), grown on demand
  void* fc_ws = nullptr;
  size_t fc_bytes = 0;
  // full-CSI-start workspace (conjugate direction, two scalars per instance), grown on demand
  void* csi_ws = nullptr;
  size_t csi_bytes = 0;
  // tile shapes of the FP32 MFMA kernels (chosen by pdf_autotune; results do not depend on them)
  int tune_ct = 2;           // column tiles per wave of the G_S^H GEMM: 1, 2 or 4
  int tune_pb = 4;           // load batch of the pixel reduction: 4 or 8
  int tune_fpp = 0;          // forward convolution: 0 half tile in place, 1 full tile with alternating row passes
  int tune_app = 0;          // adjoint convolution: likewise
  bool tuned = false;
  // optional per-kernel event timing
  bool timing = false;
  int timing_max = 0;
  std::vector<hipEvent_t> events;   // pool
  int ev_used = 0;
  std::string err_msg;
};

// Message returned by pdf_last_error(NULL).
void pdf_set_global_error(const std::string& msg);

// The stream a warm-start network was created on.
hipStream_t pdf_mlp_stream(const pdf_mlp* net);
