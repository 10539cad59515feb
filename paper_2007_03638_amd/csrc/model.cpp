#include "model.h"

#include <cstring>

namespace mera {

namespace {

constexpr int kSpins = 6, kDim = 64;

inline int bit(int state, int spin) { return (state >> (kSpins - 1 - spin)) & 1; }
inline int flip(int state, int spin) { return state ^ (1 << (kSpins - 1 - spin)); }

// out += c * X_i X_j
void add_xx(double* out, int i, int j, double c) {
  for (int y = 0; y < kDim; ++y) out[flip(flip(y, i), j) * kDim + y] += c;
}
// out += c * Y_i Y_j  (Y|b> = i (-1)^b |1-b>, so <y'|Y_i Y_j|y> = -(-1)^(b_i + b_j))
void add_yy(double* out, int i, int j, double c) {
  for (int y = 0; y < kDim; ++y) {
    double s = (bit(y, i) == bit(y, j)) ? -1.0 : 1.0;
    out[flip(flip(y, i), j) * kDim + y] += c * s;
  }
}
// out += c * Z_i Z_j
void add_zz(double* out, int i, int j, double c) {
  for (int y = 0; y < kDim; ++y) out[y * kDim + y] += c * ((bit(y, i) == bit(y, j)) ? 1.0 : -1.0);
}
// out += c * Z_i
void add_z(double* out, int i, double c) {
  for (int y = 0; y < kDim; ++y) out[y * kDim + y] += c * (bit(y, i) ? -1.0 : 1.0);
}

// hb on blocks starting at spin s (spins s..s+3), added with weight wgt
template <typename Pair, typename Field>
void add_hb(double* out, int s, double wgt, Pair pair, Field field) {
  pair(out, s + 1, s + 2, wgt);                // inter-block bond
  pair(out, s, s + 1, 0.5 * wgt);              // half of block 1 internal bond
  pair(out, s + 2, s + 3, 0.5 * wgt);          // half of block 2 internal bond
  for (int k = 0; k < 4; ++k) field(out, s + k, 0.5 * wgt);
}

}  // namespace

void build_h3_tfim(double h, double* out) {
  std::memset(out, 0, sizeof(double) * kDim * kDim);
  auto pair = [](double* o, int i, int j, double c) { add_xx(o, i, j, -c); };
  auto field = [h](double* o, int i, double c) { add_z(o, i, -h * c); };
  add_hb(out, 0, 0.5, pair, field);
  add_hb(out, 2, 0.5, pair, field);
}

void build_h3_xxz(double delta, double* out) {
  std::memset(out, 0, sizeof(double) * kDim * kDim);
  auto pair = [delta](double* o, int i, int j, double c) {
    add_xx(o, i, j, c);
    add_yy(o, i, j, c);
    add_zz(o, i, j, delta * c);
  };
  auto field = [](double*, int, double) {};
  add_hb(out, 0, 0.5, pair, field);
  add_hb(out, 2, 0.5, pair, field);
}

void build_h2_tfim(double h, double* out) {
  std::memset(out, 0, sizeof(double) * 16);
  for (int y = 0; y < 4; ++y) {
    const int b0 = (y >> 1) & 1, b1 = y & 1;
    out[(y ^ 3) * 4 + y] += -1.0;                                     // -X X
    out[y * 4 + y] += -0.5 * h * ((b0 ? -1.0 : 1.0) + (b1 ? -1.0 : 1.0));  // -h (Z 1 + 1 Z)/2
  }
}

void build_h2_xxz(double delta, double* out) {
  std::memset(out, 0, sizeof(double) * 16);
  for (int y = 0; y < 4; ++y) {
    const int b0 = (y >> 1) & 1, b1 = y & 1;
    out[(y ^ 3) * 4 + y] += 1.0 + ((b0 == b1) ? -1.0 : 1.0);          // X X + Y Y
    out[y * 4 + y] += delta * ((b0 == b1) ? 1.0 : -1.0);               // delta Z Z
  }
}

}  // namespace mera
