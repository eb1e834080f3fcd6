// Launchers of the learned-preconditioner kernels (cnn.hip).  Rows: row = cb * Ns + s, 32 channels.
#pragma once
#include "eofa_int.h"

namespace eofa {

// 4 layers; layer l maps CNN_CIN[l] -> CNN_COUT[l] live channels (padded to 32)
constexpr int CNN_LAYERS = 4;
constexpr int CNN_CIN[CNN_LAYERS] = {24, 32, 32, 32};
constexpr int CNN_COUT[CNN_LAYERS] = {32, 32, 32, 24};
constexpr int CNN_WSZ = 81 * 32 * 32;         // weights per layer (padded), [tap][n][k]
constexpr int CNN_LSZ = CNN_WSZ + 32;         // + bias
constexpr int CNN_NPARAM = CNN_LAYERS * CNN_LSZ;

hipError_t cnn_conv_fwd(const unsigned short* X, const unsigned short* W, const float* bias, void* Y, bool out_f32,
                        const Geom& g, int Ns, int relu, hipStream_t st);
int cnn_wgrad_chunks(int rows);
hipError_t cnn_wgrad(const unsigned short* dYT, const unsigned short* XT, float* part, float* gw, const Geom& g, int Ns,
                     int cin, int cout, hipStream_t st);
// part: scratch of >= 256 x 32 doubles
hipError_t cnn_bgrad(const float* dY, int rows, float* gb, int cout, double* part, hipStream_t st);
hipError_t cnn_to_chmajor(const void* in, bool in_f32, unsigned short* out, int rows, hipStream_t st);
hipError_t cnn_f32_to_bf16(const float* in, unsigned short* out, size_t n, hipStream_t st);
hipError_t cnn_relu_bwd(float* d, const unsigned short* act, size_t n, hipStream_t st);
hipError_t cnn_w_transpose(const float* w, unsigned short* wt, hipStream_t st);
hipError_t cnn_adam(float* p, const float* g, float* m, float* v, size_t n, float lr, float b1, float b2, float eps,
                    float c1, float c2, float gscale, hipStream_t st);
hipError_t cnn_half_to_rows(const cd* h, unsigned short* X, const Geom& g, int Ns, const double* scale, int inv,
                            hipStream_t st);
hipError_t cnn_half_to_rows_f32(const cd* h, float* T, const Geom& g, int Ns, const double* scale, hipStream_t st);
hipError_t cnn_rows_to_half(const float* Y, cd* h, const Geom& g, int Ns, const double* scale, hipStream_t st);
hipError_t cnn_mse(const float* Y, const float* T, float* dY, size_t n, float w, const Red& red, hipStream_t st);

}  // namespace eofa
