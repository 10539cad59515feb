// Model Hamiltonians as symmetric 3-site terms on blocked sites of two spins (host, FP64).
#pragma once

namespace mera {

// Sec. 4 cost function: TFIM local term -X_i X_{i+1} - h Z_i; XXZ term X X + Y Y + delta Z Z (Pauli units).
// Six spins s0..s5 (s0 most significant bit of the 64-dim index) form three blocked sites (s0 s1)(s2 s3)(s4 s5);
// hb on two blocks = inter-block bond + half of each block's internal bond and fields; h3 = average of hb on
// blocks (0,1) and (1,2). out: 64 x 64 row-major.
void build_h3_tfim(double h, double* out);
void build_h3_xxz(double delta, double* out);
// Two-site terms on unblocked spins for the ternary geometry: TFIM -X X - h (Z 1 + 1 Z)/2 (each site's field
// shared by its two bonds), XXZ X X + Y Y + delta Z Z. out: 4 x 4 row-major, s0 the more significant bit.
void build_h2_tfim(double h, double* out);
void build_h2_xxz(double delta, double* out);

}  // namespace mera
