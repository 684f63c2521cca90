// Internal declarations of the warm-start network (llp_cnn.hip: device kernels; llp_cnn_api.hip: host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace llp {

constexpr int kCnnLayers = 5;
constexpr int kCnnParams = 28641;  // 2*32*9+32 + 3*(32*32*9+32) + 32*9+1

// Sizes of the bands a network launch covers.
struct CnnGeom {
  int N, H, W, h, w, c;
};

int cnn_layer_cin(int l);
int cnn_layer_cout(int l);
int cnn_layer_offset(int l);   // first parameter of layer l in the flat layout (W [cout][cin][3][3], then b)
size_t cnn_tile_bytes(int cob);  // MFMA weight operands of one layer with cob blocks of 16 rows
int cnn_wgrad_parts();           // maximum workgroups (partial sums) of a weight-gradient launch
size_t cnn_wgrad_part_floats();
size_t cnn_loss_parts(const CnnGeom& g);

// Mean and std (1 where 0) of `count` arrays: out[2k], out[2k+1]; part: count * cnn_stats_parts(len) * 2
// doubles of scratch.
size_t cnn_stats_parts(size_t len);
hipError_t cnn_launch_stats(const float* src, size_t stride, size_t len, int count, double* part, float* out,
                            hipStream_t s);
// x_up and the padded 32-channel bfloat16 input planes; stats: per band (m, s), statsY: (m_Y, s_Y).
hipError_t cnn_launch_input(const CnnGeom& g, const float* X, const float* Y, const float* stats,
                            const float* statsY, float* xup, uint16_t* in0, hipStream_t s);
// One convolution layer (see k_conv): epi 0 = bias + ReLU, 1 = final (net output / z0), 2 = ReLU-derivative mask.
hipError_t cnn_launch_conv(const CnnGeom& g, int cob, int epi, const uint16_t* in, const void* wt,
                           const float* bias, uint16_t* out, const uint16_t* mask, float* netout, float* z0,
                           const float* xup, const float* stats, hipStream_t s);
// Weight and bias gradient of one layer into grad (flat layout of that layer); part: cnn_wgrad_parts() x
// cnn_wgrad_part_floats() floats of scratch.
hipError_t cnn_launch_wgrad(const CnnGeom& g, const uint16_t* gout, const uint16_t* in, float* part, int cout,
                            int cin, float* grad, hipStream_t s);
// Loss (mean squared error against t = (Z - x_up)/s) into *loss (device double) and the output gradient.
hipError_t cnn_launch_loss(const CnnGeom& g, const float* net, const float* Z, const float* xup,
                           const float* stats, uint16_t* gout, double* part, double* loss, hipStream_t s);
hipError_t cnn_launch_prep(const float* Wm, int cout, int cin, int cob, int backward, void* out, hipStream_t s);
hipError_t cnn_launch_adam(float* p, const float* grad, float* m, float* v, int n, float lr, int t, hipStream_t s);

}  // namespace llp
