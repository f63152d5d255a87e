// k_nn.h -- launchers of the convolutional stand-in for the averaging.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sedimi {

// Epilogues of the fused convolution kernel.
enum {
  EPI_FIRST = 0,  // z = conv + b; h = phi(z)
  EPI_RES = 1,    // z = conv + b; h = h_in + phi(z)
  EPI_LAST = 2,   // y = x + conv + b (FP32)
  EPI_BWD = 3     // dh = conv^T(dz) (+ dh_in); dz' = dh * phi'(z_in)
};

struct ConvGeom {
  int nx, ny, nz, ncell;
  int dil;  // dilation along z
  int neg;  // 1: negated tap offsets (data gradient)
};

struct EpiArgs {
  const __bf16* hin;  // residual input (EPI_RES: h_in; EPI_BWD: dh of the layer above)
  const __bf16* zin;  // EPI_BWD: pre-activation of the layer below
  __bf16* zout;       // EPI_FIRST/RES: pre-activation out; EPI_BWD: dz out
  __bf16* hout;       // EPI_FIRST/RES: activation out; EPI_BWD: dh out
  const float* xres;  // EPI_LAST: normalised input (global residual)
  float* yout;        // EPI_LAST: output
  float alpha;        // leaky-ReLU slope
};

struct NNNorm {
  double mean[4], std[4];
  double lw[4];  // per-channel weights of the training loss
};

// The network's skip S (the diffusion split by axis): circulant taps of the
// periodic one-dimensional steps in x and y (device FP64 arrays; tap t at
// offset off0 + t), and the z-line Thomas table (reciprocal pivots [nz],
// back-substitution multipliers [nz]) with the z coefficient c_z.
struct SplitTabs {
  const double* tapx;
  const double* tapy;
  const double* ztab;
  int off0x, ntapx, off0y, ntapy;
  double cz;
};

size_t nn_packed_elems(int cin, int cout);
void launch_conv(int cin, int cout, int epi, const ConvGeom& g, const __bf16* in,
                 const __bf16* wpk, const float* bias, const EpiArgs& e, hipStream_t s);
// Weight/bias gradients into dw [27][cin][cout], db [cout] (FP32); part must
// hold nblocks * 27 * cin * cout floats, part_b nblocks * cout.
int launch_conv_dw(int cin, int cout, const ConvGeom& g, const __bf16* x, const __bf16* dy,
                   float* part, float* part_b, float* dw, float* db, int nblocks,
                   hipStream_t s);
void launch_nn_prep(int ncell, const double* raw, const NNNorm& nm, float* xf, __bf16* xb,
                    hipStream_t s);
// out = S in on channel-last FP32 [ncell][4] fields (tmp: scratch of the same
// size); needs split_lds_bytes(nz) bytes of LDS per block (nz <= 150).
size_t split_lds_bytes(int nz);
void launch_split(int nx, int ny, int nz, int ntau, const SplitTabs& st, const float* in,
                  float* tmp, float* out, hipStream_t s);
// The network's input x - S x in BF16 (over the copy launch_nn_prep wrote).
void launch_nn_highpass(int ncell, const float* xf, const float* xs, __bf16* xb, hipStream_t s);
void launch_nn_out(int ncell, const float* y, const NNNorm& nm, double* smooth, hipStream_t s);
unsigned launch_nn_loss(int ncell, const float* y, const double* smooth, const NNNorm& nm,
                        __bf16* dy, double* part, hipStream_t s);
void launch_adam(int64_t n, float* w, float* m, float* v, const float* g, float lr, float b1,
                 float b2, float eps, int64_t t, hipStream_t s);
// Zero one layer's cross-group weights (4 groups; see sedimi_nn_set_groups).
void launch_group_mask(float* a, int cin, int cout, hipStream_t s);
void launch_pack(const float* w, int cin, int cout, __bf16* fwd, __bf16* adj, hipStream_t s);

}  // namespace sedimi
