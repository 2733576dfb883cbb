// Fourier-neural-operator stepper: device arguments and the forward launcher.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pfn {

constexpr int kC = 32;       // channel width
constexpr int kH = 128;      // hidden units of the projection
constexpr int kLayers = 4;   // Fourier layers
constexpr int kCond = 7;     // constant conditioning channels
constexpr int kMaxModes = 16;

struct FArgs {
  int nx, ny, nz, m;          // grid (nx a multiple of 32) and kept modes
  size_t nvox;
  float inv_ntot;
  uint16_t* va;               // [nvox][C] BF16 activations (ping)
  uint16_t* vb;               // [nvox][C] BF16 activations (pong)
  float* X1;                  // [nz][ny][m][2][C]
  float* X2;                  // [nz][2m][m][2][C]
  float* Y2;                  // [nz][2m][m][2][C]
  float* Y1;                  // [nz][ny][m][2][C]
  const uint16_t* wxf;        // [hi, lo][32][nx] BF16 parts of the forward x twiddles
  const uint16_t* wxi;        // [hi, lo][nx][32] BF16 parts of the scaled inverse x twiddles
  const float2* twy;
  const float2* twz;
  float lift[2 * kC];         // P0[c] (weight of f) and the folded constant K[c]
  const uint16_t* W;          // [layers][C][C] BF16 (out, in)
  const float* b;             // [layers][C]
  const uint16_t* R;          // [layers][2m][2m][m][C out][C in][re, im] BF16
  size_t r_stride;            // elements of R per layer
  const uint16_t* Q1;         // [H][C] BF16
  const float* q1;            // [H]
  const float* Q2;            // [H]
  float q2;
};

// eta_out = forward(eta_in) on stream s; eta_in and eta_out may not alias.
hipError_t forward(const FArgs& a, const float* eta_in, float* eta_out, hipStream_t s);

}  // namespace pfn
