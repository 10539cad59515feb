// Binary-MERA energy and Euclidean gradient on the GPU.
//
// Geometry (Sec. 4, binary form): w_j sends site j of layer tau to sites (2j, 2j+1) below; the disentanglers of
// a layer act on (2j+1, 2j+2). A 3-site operator on (2j, 2j+1, 2j+2) rises to (j-1, j, j+1) ("L" diagram),
// one on (2j+1, 2j+2, 2j+3) to (j, j+1, j+2) ("R" diagram); the translation average is A = (A_L + A_R)/2.
// Tensor legs: u[bl br tl tr], w[bl br t]; operators h[abc ABC] (kets lowercase).
//
// Each diagram is a pairwise contraction program (network.h). The two chi^9 steps of every diagram contract
// a 6-leg operator with the composite (u w) over two legs, then over three legs, the contraction order
// with the smallest multiply-add count for the binary 3-site maps (2 chi^9 + O(chi^8) per diagram).
//
// Energy and gradient (Sec. 4; App. B):
//   h_0 = h3, h_tau = A_tau(h_{tau-1});  rho_s = fixed point of the scale-invariant descending map;
//   e = Tr[h_T rho_s];  h~ solves <h~|(1 - A') = <h_T - e 1| with A' = A - |rho><1|;
//   D of the scale-invariant tensors = derivative of Tr[A_s(h~) rho_s] with h~, rho_s held fixed;
//   D of layer tau = derivative of Tr[A_tau(h_{tau-1}) rho_tau], rho_{tau-1} = D_tau(rho_tau).
// Each layer derivative runs one diagram forward and back (reverse accumulation with cotangent rho). Since h
// and rho are symmetric, the closed network is invariant under exchanging ket and bra, so the bra
// occurrences of u and w have the same environments as the ket ones: only ket environments are formed and
// counted twice, which with the 1/2 of the position average gives weight 1.
#include "mera_eval.h"

#include <algorithm>
#include <array>

#include <cmath>
#include <functional>

#include "linalg.h"
#include "network.h"

namespace mera {

namespace {

// Leg orders of the intermediates are chosen so that in every chi^9 step each operand is read along a
// unit-stride run: an operand read along M (or N) has its M (N) legs innermost, and when both operands are
// read along K their K legs appear in the same order in both (UWb is the bra composite stored in the order
// the descending step needs). The same holds for the K = chi^4 environment reductions of the derivative
// programs (Du, dW1, dW3): T1 and dT5 are stored with their contracted legs in the order and unit-stride leg
// of the other operand.
// The steps between "@loop" and "@end" may run in chunks of a spectator leg (h for the L diagram, e for the R
// diagram: neither is contracted by a chi^9 step) to bound the two 7-leg intermediates at large chi.
const char* const kAscL[] = {
    "W1[epEP] = w[xep] * w[xEP]",
    "W3[hrHR] = w[hyr] * w[HyR]",
    "UW[daegq] = u[daef] * w[fgq]",
    "@loop h",
    "T1[aABCgh] = h[abcABC] * u[bcgh]",
    "T2[aghHAG] = T1[aABCgh] * u[BCGH]",
    "T3[hHAGdeq] = T2[aghHAG] * UW[daegq]",
    "T4[hHeqEQ] = T3[hHAGdeq] * UW[dAEGQ]",
    "T5[hHqQpP] = T4[hHeqEQ] * W1[epEP]",
    "out[pqrPQR] += 0.5 * T5[hHqQpP] * W3[hrHR]",
    "@end",
};
const char* const kAscR[] = {
    "W1[epEP] = w[xep] * w[xEP]",
    "W3[hrHR] = w[hyr] * w[HyR]",
    "UW[cdhfq] = u[cdgh] * w[fgq]",
    "@loop e",
    "T1[cABCef] = h[abcABC] * u[abef]",
    "T2[cfeECF] = T1[cABCef] * u[ABEF]",
    "T3[eECFdhq] = T2[cfeECF] * UW[cdhfq]",
    "T4[eEhqHQ] = T3[eECFdhq] * UW[CdHFQ]",
    "T5[eEqQrR] = T4[eEhqHQ] * W3[hrHR]",
    "out[pqrPQR] += 0.5 * T5[eEqQrR] * W1[epEP]",
    "@end",
};
const char* const kDesL[] = {
    "W1[epEP] = w[xep] * w[xEP]",
    "W3[hrHR] = w[hyr] * w[HyR]",
    "UW[daegq] = u[daef] * w[fgq]",
    "UWb[dAGEQ] = u[dAEF] * w[FGQ]",
    "@loop h",
    "dT5[pqPQhH] = rho[pqrPQR] * W3[hrHR]",
    "dT4[qhHeEQ] = dT5[pqPQhH] * W1[epEP]",
    "dT3[qhHedAG] = dT4[qhHeEQ] * UWb[dAGEQ]",
    "dT2[hHAGag] = dT3[qhHedAG] * UW[daegq]",
    "dT1[hAagBC] = dT2[hHAGag] * u[BCGH]",
    "out[abcABC] += 0.5 * dT1[hAagBC] * u[bcgh]",
    "@end",
};
const char* const kDesR[] = {
    "W1[epEP] = w[xep] * w[xEP]",
    "W3[hrHR] = w[hyr] * w[HyR]",
    "UW[cdhfq] = u[cdgh] * w[fgq]",
    "UWb[dCFHQ] = u[CdGH] * w[FGQ]",
    "@loop e",
    "dT5[qrQReE] = rho[pqrPQR] * W1[epEP]",
    "dT4[qeEhHQ] = dT5[qrQReE] * W3[hrHR]",
    "dT3[qeEhdCF] = dT4[qeEhHQ] * UWb[dCFHQ]",
    "dT2[eECFcf] = dT3[qeEhdCF] * UW[cdhfq]",
    "dT1[eCcfAB] = dT2[eECFcf] * u[ABEF]",
    "out[abcABC] += 0.5 * dT1[eCcfAB] * u[abef]",
    "@end",
};
// forward of the L diagram, then reverse accumulation with cotangent rho
const char* const kGradL[] = {
    "W1[epEP] = w[xep] * w[xEP]",
    "W3[hrHR] = w[hyr] * w[HyR]",
    "UW[daegq] = u[daef] * w[fgq]",
    "UWb[dAGEQ] = u[dAEF] * w[FGQ]",
    "@zero dW1 dUW",
    "@loop h",
    "T1[BChAag] = h[abcABC] * u[bcgh]",
    "T2[aghHAG] = T1[BChAag] * u[BCGH]",
    "T3[hHAGdeq] = T2[aghHAG] * UW[daegq]",
    "T4[hHeqEQ] = T3[hHAGdeq] * UW[dAEGQ]",
    "T5[hHqQpP] = T4[hHeqEQ] * W1[epEP]",
    "dT5[pPhHqQ] = rho[pqrPQR] * W3[hrHR]",
    "dW3[hHrR] = T5[hHqQpP] * rho[pqrPQR]",
    "dT4[qhHeEQ] = dT5[pPhHqQ] * W1[epEP]",
    "dW1[eEpP] += T4[hHeqEQ] * dT5[pPhHqQ]",
    "dT3[qhHedAG] = dT4[qhHeEQ] * UWb[dAGEQ]",
    "dUW[agqed] += T2[aghHAG] * dT3[qhHedAG]",
    "dT2[hHAGag] = dT3[qhHedAG] * UW[daegq]",
    "dT1[hAagBC] = dT2[hHAGag] * u[BCGH]",
    "Du[BCGH] += T1[BChAag] * dT2[hHAGag]",
    "rhoout[abcABC] += 0.5 * dT1[hAagBC] * u[bcgh]",
    "Dw[hyr] += dW3[hHrR] * w[HyR]",
    "@end",
    "Du[daef] += dUW[agqed] * w[fgq]",
    "Dw[fgq] += u[daef] * dUW[agqed]",
    "Dw[xep] += dW1[eEpP] * w[xEP]",
};
const char* const kGradR[] = {
    "W1[epEP] = w[xep] * w[xEP]",
    "W3[hrHR] = w[hyr] * w[HyR]",
    "UW[cdhfq] = u[cdgh] * w[fgq]",
    "UWb[dCFHQ] = u[CdGH] * w[FGQ]",
    "@zero dW3 dUW",
    "@loop e",
    "T1[cABCef] = h[abcABC] * u[abef]",
    "T2[cfeECF] = T1[cABCef] * u[ABEF]",
    "T3[eECFdhq] = T2[cfeECF] * UW[cdhfq]",
    "T4[eEhqHQ] = T3[eECFdhq] * UW[CdHFQ]",
    "T5[eEqQrR] = T4[eEhqHQ] * W3[hrHR]",
    "dT5[rReEqQ] = rho[pqrPQR] * W1[epEP]",
    "dW1[eEpP] = T5[eEqQrR] * rho[pqrPQR]",
    "dT4[qeEhHQ] = dT5[rReEqQ] * W3[hrHR]",
    "dW3[hHrR] += T4[eEhqHQ] * dT5[rReEqQ]",
    "dT3[qeEhdCF] = dT4[qeEhHQ] * UWb[dCFHQ]",
    "dUW[cfqhd] += T2[cfeECF] * dT3[qeEhdCF]",
    "dT2[eECFcf] = dT3[qeEhdCF] * UW[cdhfq]",
    "dT1[eCcfAB] = dT2[eECFcf] * u[ABEF]",
    "Du[ABEF] += T1[cABCef] * dT2[eECFcf]",
    "rhoout[abcABC] += 0.5 * dT1[eCcfAB] * u[abef]",
    "Dw[xep] += dW1[eEpP] * w[xEP]",
    "@end",
    "Du[cdgh] += dUW[cfqhd] * w[fgq]",
    "Dw[fgq] += u[cdgh] * dUW[cfqhd]",
    "Dw[hyr] += dW3[hHrR] * w[HyR]",
};
// The same two derivative programs split into a forward half, which also produces the layer's ascended operator,
// and a reverse half. The forward half keeps the activations the reverse half reads (F1, F2, F4, F5: a^6, a^6,
// a^4 b^2 and a^2 b^4 elements) in caller buffers, so a transition layer's forward pass, which its ascending map
// computes anyway, is not repeated in its derivative.
const char* const kFwdL[] = {
    "W1[epEP] = w[xep] * w[xEP]",
    "W3[hrHR] = w[hyr] * w[HyR]",
    "UW[daegq] = u[daef] * w[fgq]",
    "@loop h",
    "F1[BChAag] = h[abcABC] * u[bcgh]",
    "F2[aghHAG] = F1[BChAag] * u[BCGH]",
    "T3[hHAGdeq] = F2[aghHAG] * UW[daegq]",
    "F4[hHeqEQ] = T3[hHAGdeq] * UW[dAEGQ]",
    "F5[hHqQpP] = F4[hHeqEQ] * W1[epEP]",
    "out[pqrPQR] += 0.5 * F5[hHqQpP] * W3[hrHR]",
    "@end",
};
const char* const kRevL[] = {
    "W1[epEP] = w[xep] * w[xEP]",
    "W3[hrHR] = w[hyr] * w[HyR]",
    "UW[daegq] = u[daef] * w[fgq]",
    "UWb[dAGEQ] = u[dAEF] * w[FGQ]",
    "@zero dW1 dUW",
    "@loop h",
    "dT5[pPhHqQ] = rho[pqrPQR] * W3[hrHR]",
    "dW3[hHrR] = F5[hHqQpP] * rho[pqrPQR]",
    "dT4[qhHeEQ] = dT5[pPhHqQ] * W1[epEP]",
    "dW1[eEpP] += F4[hHeqEQ] * dT5[pPhHqQ]",
    "dT3[qhHedAG] = dT4[qhHeEQ] * UWb[dAGEQ]",
    "dUW[agqed] += F2[aghHAG] * dT3[qhHedAG]",
    "dT2[hHAGag] = dT3[qhHedAG] * UW[daegq]",
    "dT1[hAagBC] = dT2[hHAGag] * u[BCGH]",
    "Du[BCGH] += F1[BChAag] * dT2[hHAGag]",
    "rhoout[abcABC] += 0.5 * dT1[hAagBC] * u[bcgh]",
    "Dw[hyr] += dW3[hHrR] * w[HyR]",
    "@end",
    "Du[daef] += dUW[agqed] * w[fgq]",
    "Dw[fgq] += u[daef] * dUW[agqed]",
    "Dw[xep] += dW1[eEpP] * w[xEP]",
};
const char* const kFwdR[] = {
    "W1[epEP] = w[xep] * w[xEP]",
    "W3[hrHR] = w[hyr] * w[HyR]",
    "UW[cdhfq] = u[cdgh] * w[fgq]",
    "@loop e",
    "F1[cABCef] = h[abcABC] * u[abef]",
    "F2[cfeECF] = F1[cABCef] * u[ABEF]",
    "T3[eECFdhq] = F2[cfeECF] * UW[cdhfq]",
    "F4[eEhqHQ] = T3[eECFdhq] * UW[CdHFQ]",
    "F5[eEqQrR] = F4[eEhqHQ] * W3[hrHR]",
    "out[pqrPQR] += 0.5 * F5[eEqQrR] * W1[epEP]",
    "@end",
};
const char* const kRevR[] = {
    "W1[epEP] = w[xep] * w[xEP]",
    "W3[hrHR] = w[hyr] * w[HyR]",
    "UW[cdhfq] = u[cdgh] * w[fgq]",
    "UWb[dCFHQ] = u[CdGH] * w[FGQ]",
    "@zero dW3 dUW",
    "@loop e",
    "dT5[rReEqQ] = rho[pqrPQR] * W1[epEP]",
    "dW1[eEpP] = F5[eEqQrR] * rho[pqrPQR]",
    "dT4[qeEhHQ] = dT5[rReEqQ] * W3[hrHR]",
    "dW3[hHrR] += F4[eEhqHQ] * dT5[rReEqQ]",
    "dT3[qeEhdCF] = dT4[qeEhHQ] * UWb[dCFHQ]",
    "dUW[cfqhd] += F2[cfeECF] * dT3[qeEhdCF]",
    "dT2[eECFcf] = dT3[qeEhdCF] * UW[cdhfq]",
    "dT1[eCcfAB] = dT2[eECFcf] * u[ABEF]",
    "Du[ABEF] += F1[cABCef] * dT2[eECFcf]",
    "rhoout[abcABC] += 0.5 * dT1[eCcfAB] * u[abef]",
    "Dw[xep] += dW1[eEpP] * w[xEP]",
    "@end",
    "Du[cdgh] += dUW[cfqhd] * w[fgq]",
    "Dw[fgq] += u[cdgh] * dUW[cfqhd]",
    "Dw[hyr] += dW3[hHrR] * w[HyR]",
};
// reduced density matrix on the two top legs of u from the two-site marginal above (Sec. 4, rho_v)
const char* const kRhoU[] = {
    "Z1[epEP] = w[xep] * w[xEP]",
    "Z3[fqFQ] = w[fyq] * w[FyQ]",
    "R1[eEqQ] = Z1[epEP] * rho2[pqPQ]",
    "rhou[efEF] = R1[eEqQ] * Z3[fqFQ]",
};

// ---- ternary MERA with two-site operators (Sec. 4, the paper's benchmark geometry) ---------------------------
// w[x y z t] covers the sites (3k, 3k+1, 3k+2) below and maps to site k above; u[bl br tl tr] acts on
// (3k+2, 3k+3). A two-site operator h[ab AB] on (3k, 3k+1), (3k+1, 3k+2) or (3k+2, 3k+3) rises through the L, C or R
// diagram; A = (A_L + A_C + A_R)/3. Legs p, q, P, Q are top legs (b), all others bottom legs (a). Each diagram
// costs O(a^8).
const char* const kTAscL[] = {
    "Wl[fpFP] = w[xyfp] * w[xyFP]",
    "Wr[cbqCBQ] = w[cbzq] * w[CBzQ]",
    "U[afcAFC] = u[eafc] * u[eAFC]",
    "T1[bBfcFC] = h[abAB] * U[afcAFC]",
    "T2[bBcCpP] = T1[bBfcFC] * Wl[fpFP]",
    "out[pqPQ] += 0.3333333333333333 * T2[bBcCpP] * Wr[cbqCBQ]",
};
const char* const kTAscC[] = {
    "Wl[acpACP] = w[xacp] * w[xACP]",
    "Wr[fqFQ] = w[fyzq] * w[FyzQ]",
    "U[bcfBCF] = u[becf] * u[BeCF]",
    "T1[aAcfCF] = h[abAB] * U[bcfBCF]",
    "T2[aAcCqQ] = T1[aAcfCF] * Wr[fqFQ]",
    "out[pqPQ] += 0.3333333333333333 * T2[aAcCqQ] * Wl[acpACP]",
};
const char* const kTAscR[] = {
    "Wl[cpCP] = w[xycp] * w[xyCP]",
    "Wr[dqDQ] = w[dzvq] * w[DzvQ]",
    "T1[ABcd] = h[abAB] * u[abcd]",
    "T2[cdCD] = T1[ABcd] * u[ABCD]",
    "T3[dDpP] = T2[cdCD] * Wl[cpCP]",
    "out[pqPQ] += 0.3333333333333333 * T3[dDpP] * Wr[dqDQ]",
};
const char* const kTDesL[] = {
    "Wl[fpFP] = w[xyfp] * w[xyFP]",
    "Wr[cbqCBQ] = w[cbzq] * w[CBzQ]",
    "U[afcAFC] = u[eafc] * u[eAFC]",
    "R1[pPbBcC] = rho[pqPQ] * Wr[cbqCBQ]",
    "R2[bBfcFC] = R1[pPbBcC] * Wl[fpFP]",
    "out[abAB] += 0.3333333333333333 * R2[bBfcFC] * U[afcAFC]",
};
const char* const kTDesC[] = {
    "Wl[acpACP] = w[xacp] * w[xACP]",
    "Wr[fqFQ] = w[fyzq] * w[FyzQ]",
    "U[bcfBCF] = u[becf] * u[BeCF]",
    "R1[qQacAC] = rho[pqPQ] * Wl[acpACP]",
    "R2[acACfF] = R1[qQacAC] * Wr[fqFQ]",
    "out[abAB] += 0.3333333333333333 * R2[acACfF] * U[bcfBCF]",
};
const char* const kTDesR[] = {
    "Wl[cpCP] = w[xycp] * w[xyCP]",
    "Wr[dqDQ] = w[dzvq] * w[DzvQ]",
    "R1[qQcC] = rho[pqPQ] * Wl[cpCP]",
    "R2[cCdD] = R1[qQcC] * Wr[dqDQ]",
    "R3[cdAB] = R2[cCdD] * u[ABCD]",
    "out[abAB] += 0.3333333333333333 * R3[cdAB] * u[abcd]",
};
// Environments of the ket copies of u, of the left and of the right isometry (the bra copies give the same by the
// symmetry of h and rho, hence the weight 2/3), and the descended rho, for one diagram.
const char* const kTGradL[] = {
    "Wl[fpFP] = w[xyfp] * w[xyFP]",
    "Wr[cbqCBQ] = w[cbzq] * w[CBzQ]",
    "U[afcAFC] = u[eafc] * u[eAFC]",
    "T1[bBfcFC] = h[abAB] * U[afcAFC]",
    "T2[bBcCpP] = T1[bBfcFC] * Wl[fpFP]",
    "R1[pPbBcC] = rho[pqPQ] * Wr[cbqCBQ]",
    "R2[bBfcFC] = R1[pPbBcC] * Wl[fpFP]",
    "X1[acfAFC] = h[abAB] * R2[bBfcFC]",
    "Du[eafc] += 0.6666666666666666 * X1[acfAFC] * u[eAFC]",
    "Mwl[fFpP] = T1[bBfcFC] * R1[pPbBcC]",
    "Dw[xyfp] += 0.6666666666666666 * w[xyFP] * Mwl[fFpP]",
    "Mwr[bBcCqQ] = T2[bBcCpP] * rho[pqPQ]",
    "Dw[cbzq] += 0.6666666666666666 * Mwr[bBcCqQ] * w[CBzQ]",
    "rhoout[abAB] += 0.3333333333333333 * R2[bBfcFC] * U[afcAFC]",
};
const char* const kTGradC[] = {
    "Wl[acpACP] = w[xacp] * w[xACP]",
    "Wr[fqFQ] = w[fyzq] * w[FyzQ]",
    "U[bcfBCF] = u[becf] * u[BeCF]",
    "R1[qQacAC] = rho[pqPQ] * Wl[acpACP]",
    "R2[acACfF] = R1[qQacAC] * Wr[fqFQ]",
    "rhoout[abAB] += 0.3333333333333333 * R2[acACfF] * U[bcfBCF]",
    "X1[bBcCfF] = h[abAB] * R2[acACfF]",
    "Du[becf] += 0.6666666666666666 * X1[bBcCfF] * u[BeCF]",
    "T1[aAcfCF] = h[abAB] * U[bcfBCF]",
    "T2[aAcCqQ] = T1[aAcfCF] * Wr[fqFQ]",
    "Mwl[aAcCpP] = T2[aAcCqQ] * rho[pqPQ]",
    "Dw[xacp] += 0.6666666666666666 * w[xACP] * Mwl[aAcCpP]",
    "Mwr[fFqQ] = T1[aAcfCF] * R1[qQacAC]",
    "Dw[fyzq] += 0.6666666666666666 * Mwr[fFqQ] * w[FyzQ]",
};
const char* const kTGradR[] = {
    "Wl[cpCP] = w[xycp] * w[xyCP]",
    "Wr[dqDQ] = w[dzvq] * w[DzvQ]",
    "R1[qQcC] = rho[pqPQ] * Wl[cpCP]",
    "R2[cCdD] = R1[qQcC] * Wr[dqDQ]",
    "R3[cdAB] = R2[cCdD] * u[ABCD]",
    "rhoout[abAB] += 0.3333333333333333 * R3[cdAB] * u[abcd]",
    "Du[abcd] += 0.6666666666666666 * h[abAB] * R3[cdAB]",
    "T1[ABcd] = h[abAB] * u[abcd]",
    "T2[cdCD] = T1[ABcd] * u[ABCD]",
    "T3[cCqQ] = T2[cdCD] * Wr[dqDQ]",
    "Mwl[cCpP] = T3[cCqQ] * rho[pqPQ]",
    "Dw[xycp] += 0.6666666666666666 * w[xyCP] * Mwl[cCpP]",
    "Mwr[dDqQ] = T2[cdCD] * R1[qQcC]",
    "Dw[dzvq] += 0.6666666666666666 * Mwr[dDqQ] * w[DzvQ]",
};
// density matrix on the two top legs of u: the top two-site rho pushed down through w_k (x) w_{k+1}
const char* const kTRhoU[] = {
    "Wl[cpCP] = w[xycp] * w[xyCP]",
    "Wr[dqDQ] = w[dzvq] * w[DzvQ]",
    "R1[qQcC] = rho2[pqPQ] * Wl[cpCP]",
    "rhou[cdCD] = R1[qQcC] * Wr[dqDQ]",
};

template <size_t N>
std::vector<std::string> lines(const char* const (&a)[N]) {
  return std::vector<std::string>(a, a + N);
}

struct Programs {
  Program asc[2], des[2], grad[2], fwd[2], rev[2], rhou;
  Program tasc[3], tdes[3], tgrad[3], trhou;  // ternary geometry
  Programs() {
    const std::vector<std::string> ext = {"h",  "u",    "w",    "rho", "out", "Du", "Dw", "rhoout",
                                          "rho2", "rhou", "F1",  "F2",  "F4",  "F5"};
    asc[0] = Program::parse("ascL", lines(kAscL), ext);
    asc[1] = Program::parse("ascR", lines(kAscR), ext);
    des[0] = Program::parse("desL", lines(kDesL), ext);
    des[1] = Program::parse("desR", lines(kDesR), ext);
    grad[0] = Program::parse("gradL", lines(kGradL), ext);
    grad[1] = Program::parse("gradR", lines(kGradR), ext);
    fwd[0] = Program::parse("fwdL", lines(kFwdL), ext);
    fwd[1] = Program::parse("fwdR", lines(kFwdR), ext);
    rev[0] = Program::parse("revL", lines(kRevL), ext);
    rev[1] = Program::parse("revR", lines(kRevR), ext);
    rhou = Program::parse("rhou", lines(kRhoU), ext);
    tasc[0] = Program::parse("tascL", lines(kTAscL), ext);
    tasc[1] = Program::parse("tascC", lines(kTAscC), ext);
    tasc[2] = Program::parse("tascR", lines(kTAscR), ext);
    tdes[0] = Program::parse("tdesL", lines(kTDesL), ext);
    tdes[1] = Program::parse("tdesC", lines(kTDesC), ext);
    tdes[2] = Program::parse("tdesR", lines(kTDesR), ext);
    tgrad[0] = Program::parse("tgradL", lines(kTGradL), ext);
    tgrad[1] = Program::parse("tgradC", lines(kTGradC), ext);
    tgrad[2] = Program::parse("tgradR", lines(kTGradR), ext);
    trhou = Program::parse("trhou", lines(kTRhoU), ext);
    // the chi^9 (binary) and chi^8 (ternary) networks are worth grouping across concurrent jobs
    for (Program* p : {&asc[0], &asc[1], &des[0], &des[1], &grad[0], &grad[1], &fwd[0], &fwd[1], &rev[0], &rev[1],
                       &tasc[0], &tasc[1], &tasc[2], &tdes[0], &tdes[1], &tdes[2], &tgrad[0], &tgrad[1], &tgrad[2]})
      p->batch = true;
  }
};

const Programs& programs() {
  static const Programs p;
  return p;
}

LegDims legs(int a, int b) {
  LegDims d;
  d.fill(0);
  for (char c : std::string("abcdefghxyABCEFGH")) d[(unsigned char)c] = a;
  for (char c : std::string("pqrPQR")) d[(unsigned char)c] = b;
  return d;
}

int64_t p6(int64_t x) { return x * x * x * x * x * x; }

// leg extents of the ternary programs: p, q, P, Q are top legs
LegDims legs_ternary(int a, int b) {
  LegDims d;
  d.fill(0);
  for (char c : std::string("abcdefvxyzABCDF")) d[(unsigned char)c] = a;
  for (char c : std::string("pqPQ")) d[(unsigned char)c] = b;
  return d;
}

LegDims legs_of(const LayerDim& L) { return L.ternary ? legs_ternary(L.a, L.b) : legs(L.a, L.b); }

// Chunk of the loop leg for the 7-leg intermediates (a^6 b elements each): whole when they fit the context's
// limit, else the largest divisor of a keeping each chunked one within half of it.
int64_t loop_chunk(const Ctx& ctx, const LayerDim& L, size_t eb) {
  if (L.ternary) return 0;  // the ternary networks have no loop; their intermediates are at most a^6
  const double full = (double)p6(L.a) * L.b * eb;
  const double lim = (double)ctx.inter_limit;
  if (full <= lim) return 0;
  const double per = full / L.a;
  for (int64_t c = L.a; c >= 1; --c)
    if (L.a % c == 0 && per * c <= 0.5 * lim) return c;
  return 1;
}

// Device element pointers of the contraction precision for one layer's tensors.
struct LayerTensors {
  void* u;
  void* w;
};

}  // namespace

std::vector<LayerDim> layer_dims(const mera_shape& s) {
  MERA_CHECK(s.T >= 1 && s.d >= 2 && s.chi >= 2, MERA_EINVAL, "shape: need T >= 1, d >= 2, chi >= 2");
  MERA_CHECK(s.geometry == 0 || s.geometry == 1, MERA_EINVAL, "shape: geometry must be 0 (binary) or 1 (ternary)");
  const bool ter = s.geometry == 1;
  std::vector<LayerDim> out;
  int a = s.d;
  for (int t = 0; t < s.T; ++t) {
    const int64_t fan = ter ? (int64_t)a * a * a : (int64_t)a * a;
    int b = (int)std::min<int64_t>((int64_t)s.chi, fan);
    out.push_back({a, b, ter});
    a = b;
  }
  MERA_CHECK(a == s.chi, MERA_EINVAL,
             "top transition dimension " + std::to_string(a) + " != chi " + std::to_string(s.chi));
  out.push_back({s.chi, s.chi, ter});
  return out;
}

int default_krylov_dim(size_t vector_bytes) {
  const double fit = (double)((size_t)16 << 30) / (double)vector_bytes - 1.0;  // basis of dim + 1 vectors
  return (int)std::max(4.0, std::min(16.0, std::floor(fit)));
}

size_t activation_cache_bytes(const std::vector<LayerDim>& dims, size_t eb) {
  if (dims.empty() || dims[0].ternary) return 0;
  size_t bytes = 0;
  for (size_t t = 0; t + 1 < dims.size(); ++t) {
    const int64_t a = dims[t].a, b = dims[t].b;
    bytes += 2 * eb * (size_t)(2 * a * a * a * a * a * a + a * a * a * a * b * b + a * a * b * b * b * b);
  }
  return bytes;
}

namespace {

// diagrams of one layer map: the L/R pair (binary) or L/C/R (ternary)
int n_diagrams(const LayerDim& L) { return L.ternary ? 3 : 2; }
const Program& asc_prog(const LayerDim& L, int s) { return L.ternary ? programs().tasc[s] : programs().asc[s]; }
const Program& des_prog(const LayerDim& L, int s) { return L.ternary ? programs().tdes[s] : programs().des[s]; }
const Program& grad_prog(const LayerDim& L, int s) { return L.ternary ? programs().tgrad[s] : programs().grad[s]; }

void ascend_raw(Ctx& ctx, const LayerDim& L, LayerTensors t, VPtr in, VPtr out, Prec prec) {
  fill(ctx, out, L.opsize(L.b), 0.0);
  const LegDims d = legs_of(L);
  const int64_t ch = loop_chunk(ctx, L, elem_bytes(prec));
  for (int s = 0; s < n_diagrams(L); ++s)
    run_program(ctx, asc_prog(L, s), d, {{"h", in.p}, {"u", t.u}, {"w", t.w}, {"out", out.p}}, prec, ch);
  symmetrize(ctx, out, L.opdim(L.b));
}

void descend_raw(Ctx& ctx, const LayerDim& L, LayerTensors t, VPtr in, VPtr out, Prec prec) {
  fill(ctx, out, L.opsize(L.a), 0.0);
  const LegDims d = legs_of(L);
  const int64_t ch = loop_chunk(ctx, L, elem_bytes(prec));
  for (int s = 0; s < n_diagrams(L); ++s)
    run_program(ctx, des_prog(L, s), d, {{"rho", in.p}, {"u", t.u}, {"w", t.w}, {"out", out.p}}, prec, ch);
  symmetrize(ctx, out, L.opdim(L.a));
}

// D_u, D_w (+)= derivative of Tr[A(h) rho]; rhoout = D(rho). Du, Dw, rhoout are overwritten.
void layer_grad(Ctx& ctx, const LayerDim& L, LayerTensors t, VPtr h, VPtr rho, VPtr Du, VPtr Dw, VPtr rhoout,
                Prec prec) {
  const int64_t a2 = (int64_t)L.a * L.a;
  fill(ctx, Du, a2 * a2, 0.0);
  fill(ctx, Dw, L.wrows() * L.b, 0.0);
  fill(ctx, rhoout, L.opsize(L.a), 0.0);
  const LegDims d = legs_of(L);
  const int64_t ch = loop_chunk(ctx, L, elem_bytes(prec));
  for (int s = 0; s < n_diagrams(L); ++s)
    run_program(ctx, grad_prog(L, s), d,
                {{"h", h.p}, {"rho", rho.p}, {"u", t.u}, {"w", t.w}, {"Du", Du.p}, {"Dw", Dw.p},
                 {"rhoout", rhoout.p}},
                prec, ch);
  symmetrize(ctx, rhoout, L.opdim(L.a));
}

// Caller buffers of the forward activations of one transition layer, per diagram: F1, F2, F4, F5.
struct Activations {
  void* F[2][4] = {};
};

// Element counts of F1, F2, F4, F5 (the same for both diagrams).
std::array<int64_t, 4> activation_elems(const LayerDim& L) {
  const int64_t a = L.a, b = L.b;
  return {a * a * a * a * a * a, a * a * a * a * a * a, a * a * a * a * b * b, a * a * b * b * b * b};
}

// Ascending map of a binary transition layer through the forward halves of its derivative programs, keeping the
// activations for layer_grad_rev.
void ascend_fwd(Ctx& ctx, const LayerDim& L, LayerTensors t, VPtr in, VPtr out, Prec prec, const Activations& act) {
  fill(ctx, out, L.opsize(L.b), 0.0);
  const LegDims d = legs_of(L);
  const int64_t ch = loop_chunk(ctx, L, elem_bytes(prec));
  for (int s = 0; s < 2; ++s)
    run_program(ctx, programs().fwd[s], d,
                {{"h", in.p}, {"u", t.u}, {"w", t.w}, {"out", out.p}, {"F1", act.F[s][0]}, {"F2", act.F[s][1]},
                 {"F4", act.F[s][2]}, {"F5", act.F[s][3]}},
                prec, ch);
  symmetrize(ctx, out, L.opdim(L.b));
}

// layer_grad from the activations ascend_fwd kept (the reverse halves only).
void layer_grad_rev(Ctx& ctx, const LayerDim& L, LayerTensors t, VPtr rho, VPtr Du, VPtr Dw, VPtr rhoout, Prec prec,
                    const Activations& act) {
  const int64_t a2 = (int64_t)L.a * L.a;
  fill(ctx, Du, a2 * a2, 0.0);
  fill(ctx, Dw, L.wrows() * L.b, 0.0);
  fill(ctx, rhoout, L.opsize(L.a), 0.0);
  const LegDims d = legs_of(L);
  const int64_t ch = loop_chunk(ctx, L, elem_bytes(prec));
  for (int s = 0; s < 2; ++s)
    run_program(ctx, programs().rev[s], d,
                {{"rho", rho.p}, {"u", t.u}, {"w", t.w}, {"Du", Du.p}, {"Dw", Dw.p}, {"rhoout", rhoout.p},
                 {"F1", act.F[s][0]}, {"F2", act.F[s][1]}, {"F4", act.F[s][2]}, {"F5", act.F[s][3]}},
                prec, ch);
  symmetrize(ctx, rhoout, L.opdim(L.a));
}

struct KStat {
  int apps = 0;
  double res = 0.0;
  bool converged = false;
};

// Restarted GMRES(m) for op(x) = b, starting from x (in/out). Vectors of length n in precision `prec`,
// scalars in FP64; classical Gram-Schmidt applied twice; restart residual from the Arnoldi relation. Within an
// Arnoldi step the projection coefficients and the new vector's norm stay in device memory (the operator, too,
// must not synchronise); one copy to the host per step brings them back for the Hessenberg matrix.
KStat gmres(Ctx& ctx, const std::function<void(VPtr, VPtr)>& op, VPtr b, VPtr x, int64_t n, int m, double tol,
            int max_restarts, Prec prec, const char* label) {
  KStat st;
  const size_t bytes = (size_t)n * elem_bytes(prec);
  std::vector<VPtr> V(m + 1);
  for (int i = 0; i <= m; ++i) V[i] = VPtr{ctx.buf("krylov.v" + std::to_string(i), bytes), prec};
  VPtr R{ctx.buf("krylov.r", bytes), prec};
  const double bnorm = nrm2(ctx, b, n);
  MERA_CHECK(std::isfinite(bnorm), MERA_ENONFINITE, "non-finite right-hand side in Krylov solve");
  if (bnorm == 0.0) {
    fill(ctx, x, n, 0.0);
    st.converged = true;
    return st;
  }
  op(x, V[0]);
  st.apps++;
  axpby(ctx, 1.0, b, -1.0, V[0], n);  // V0 = b - A x
  double beta = nrm2(ctx, V[0], n);
  MERA_CHECK(std::isfinite(beta), MERA_ENONFINITE, "non-finite residual in Krylov solve");
  std::vector<double> H((m + 1) * m), Hr((m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  // device scalars of one Arnoldi step: two passes of projection coefficients, the norm, a work slot
  double* dsc = static_cast<double*>(ctx.buf("krylov.scalars", (size_t)(2 * (m + 1) + 2) * sizeof(double)));
  double* dh1 = dsc;
  double* dh2 = dsc + (m + 1);
  double* dhn = dsc + 2 * (m + 1);
  std::vector<double> hsc(2 * (m + 1) + 2);
  for (int restart = 0; restart <= max_restarts; ++restart) {
    st.res = beta / bnorm;
    if (ctx.verbose > 0) {
      std::fprintf(stderr, "[mera] %s solve: restart %d, %d applications, relative residual %.3e\n", label, restart,
                   st.apps, st.res);
      std::fflush(stderr);
    }
    if (beta <= tol * bnorm) {
      st.converged = true;
      break;
    }
    if (restart == max_restarts) break;
    scal(ctx, 1.0 / beta, V[0], n);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    for (int j = 0; j < m; ++j) {
      op(V[j], V[j + 1]);
      st.apps++;
      // classical Gram-Schmidt, twice: each pass is one fused projection onto V_0..V_j and one fused update
      multi_dot_dev(ctx, V.data(), j + 1, V[j + 1], n, dh1);
      multi_axpby_dev(ctx, V.data(), dh1, -1.0, j + 1, 1.0, V[j + 1], n);
      multi_dot_dev(ctx, V.data(), j + 1, V[j + 1], n, dh2);
      multi_axpby_dev(ctx, V.data(), dh2, -1.0, j + 1, 1.0, V[j + 1], n);
      normalize_dev(ctx, V[j + 1], n, dhn, dhn + 1);
      MERA_HIP(hipMemcpyAsync(hsc.data(), dsc, hsc.size() * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
      ctx.sync();
      for (int i = 0; i <= j; ++i) {
        H[i * m + j] += hsc[i];
        H[i * m + j] += hsc[(m + 1) + i];
      }
      const double hn = hsc[2 * (m + 1)];
      MERA_CHECK(std::isfinite(hn), MERA_ENONFINITE, "non-finite Krylov vector");
      H[(j + 1) * m + j] = hn;
      // rotated copy for the least-squares solve
      for (int i = 0; i <= j + 1; ++i) Hr[i * m + j] = H[i * m + j];
      for (int i = 0; i < j; ++i) {
        double t0 = cs[i] * Hr[i * m + j] + sn[i] * Hr[(i + 1) * m + j];
        double t1 = -sn[i] * Hr[i * m + j] + cs[i] * Hr[(i + 1) * m + j];
        Hr[i * m + j] = t0;
        Hr[(i + 1) * m + j] = t1;
      }
      double den = std::hypot(Hr[j * m + j], Hr[(j + 1) * m + j]);
      cs[j] = den > 0 ? Hr[j * m + j] / den : 1.0;
      sn[j] = den > 0 ? Hr[(j + 1) * m + j] / den : 0.0;
      Hr[j * m + j] = den;
      Hr[(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      k = j + 1;
      if (std::fabs(g[j + 1]) <= tol * bnorm || hn == 0.0) break;
    }
    // back substitution
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int l = i + 1; l < k; ++l) s -= Hr[i * m + l] * y[l];
      y[i] = s / Hr[i * m + i];
    }
    multi_axpby(ctx, V.data(), y.data(), k, 1.0, x, n);
    // residual r = V_{0..k} (beta e1 - Hbar y)
    std::vector<double> c(k + 1, 0.0);
    c[0] = beta;
    for (int i = 0; i <= k; ++i)
      for (int l = 0; l < k; ++l) c[i] -= H[i * m + l] * y[l];
    multi_axpby(ctx, V.data(), c.data(), k + 1, 0.0, R, n);
    std::swap(V[0], R);
    beta = nrm2(ctx, V[0], n);
    MERA_CHECK(std::isfinite(beta), MERA_ENONFINITE, "non-finite residual in Krylov solve");
  }
  // keep the scratch names stable for the next call (V[0] may have been swapped with R)
  return st;
}

}  // namespace

void ascend_op(Ctx& ctx, const LayerDim& L, const double* u, const double* w, Prec prec, const double* hin,
               double* hout) {
  const int64_t a2 = (int64_t)L.a * L.a;
  if (prec == Prec::F64) {
    ascend_raw(ctx, L, {(void*)u, (void*)w}, VPtr{(void*)hin, prec}, VPtr{hout, prec}, prec);
    return;
  }
  void* us = ctx.buf("op.u", a2 * a2 * 4);
  void* ws = ctx.buf("op.w", L.wrows() * L.b * 4);
  void* hi = ctx.buf("op.in", L.opsize(L.a) * 4);
  void* ho = ctx.buf("op.out", L.opsize(L.b) * 4);
  copy(ctx, VPtr{us, prec}, VPtr{(void*)u, Prec::F64}, a2 * a2);
  copy(ctx, VPtr{ws, prec}, VPtr{(void*)w, Prec::F64}, L.wrows() * L.b);
  copy(ctx, VPtr{hi, prec}, VPtr{(void*)hin, Prec::F64}, L.opsize(L.a));
  ascend_raw(ctx, L, {us, ws}, VPtr{hi, prec}, VPtr{ho, prec}, prec);
  copy(ctx, VPtr{hout, Prec::F64}, VPtr{ho, prec}, L.opsize(L.b));
}

void descend_op(Ctx& ctx, const LayerDim& L, const double* u, const double* w, Prec prec, const double* rin,
                double* rout) {
  const int64_t a2 = (int64_t)L.a * L.a;
  if (prec == Prec::F64) {
    descend_raw(ctx, L, {(void*)u, (void*)w}, VPtr{(void*)rin, prec}, VPtr{rout, prec}, prec);
    return;
  }
  void* us = ctx.buf("op.u", a2 * a2 * 4);
  void* ws = ctx.buf("op.w", L.wrows() * L.b * 4);
  void* ri = ctx.buf("op.in", L.opsize(L.b) * 4);
  void* ro = ctx.buf("op.out", L.opsize(L.a) * 4);
  copy(ctx, VPtr{us, prec}, VPtr{(void*)u, Prec::F64}, a2 * a2);
  copy(ctx, VPtr{ws, prec}, VPtr{(void*)w, Prec::F64}, L.wrows() * L.b);
  copy(ctx, VPtr{ri, prec}, VPtr{(void*)rin, Prec::F64}, L.opsize(L.b));
  descend_raw(ctx, L, {us, ws}, VPtr{ri, prec}, VPtr{ro, prec}, prec);
  copy(ctx, VPtr{rout, Prec::F64}, VPtr{ro, prec}, L.opsize(L.a));
}

void layer_grad_op(Ctx& ctx, const LayerDim& L, const double* u, const double* w, Prec prec, bool split,
                   const double* hin, const double* rin, double* hout, double* Du, double* Dw, double* rout) {
  MERA_CHECK(!split || !L.ternary, MERA_EINVAL, "the split forward/reverse programs exist for the binary geometry");
  MERA_CHECK(split || hout == nullptr, MERA_EINVAL, "h_out is produced only by the split programs");
  const int64_t a2 = (int64_t)L.a * L.a;
  const int64_t wn = L.wrows() * L.b;
  const size_t eb = elem_bytes(prec);
  LayerTensors t{(void*)u, (void*)w};
  VPtr hi{(void*)hin, prec}, ri{(void*)rin, prec};
  VPtr du{Du, prec}, dw{Dw, prec};
  if (prec != Prec::F64) {
    t.u = ctx.buf("op.u", a2 * a2 * 4);
    t.w = ctx.buf("op.w", wn * 4);
    hi = VPtr{ctx.buf("op.in", L.opsize(L.a) * 4), prec};
    ri = VPtr{ctx.buf("op.in2", L.opsize(L.b) * 4), prec};
    du = VPtr{ctx.buf("Dacc.u", a2 * a2 * 4), prec};
    dw = VPtr{ctx.buf("Dacc.w", wn * 4), prec};
    copy(ctx, VPtr{t.u, prec}, VPtr{(void*)u, Prec::F64}, a2 * a2);
    copy(ctx, VPtr{t.w, prec}, VPtr{(void*)w, Prec::F64}, wn);
    copy(ctx, hi, VPtr{(void*)hin, Prec::F64}, L.opsize(L.a));
    copy(ctx, ri, VPtr{(void*)rin, Prec::F64}, L.opsize(L.b));
  }
  VPtr ro{ctx.buf("op.out", L.opsize(L.a) * eb), prec};
  if (split) {
    VPtr ho{ctx.buf("op.out2", L.opsize(L.b) * eb), prec};
    Activations act;
    const auto n = activation_elems(L);
    for (int s = 0; s < 2; ++s)
      for (int j = 0; j < 4; ++j)
        act.F[s][j] = ctx.buf("act.op." + std::to_string(s) + "." + std::to_string(j), (size_t)n[j] * eb);
    ascend_fwd(ctx, L, t, hi, ho, prec, act);
    layer_grad_rev(ctx, L, t, ri, du, dw, ro, prec, act);
    if (hout) copy(ctx, VPtr{hout, Prec::F64}, ho, L.opsize(L.b));
  } else {
    layer_grad(ctx, L, t, hi, ri, du, dw, ro, prec);
  }
  if (prec != Prec::F64) {
    copy(ctx, VPtr{Du, Prec::F64}, du, a2 * a2);
    copy(ctx, VPtr{Dw, Prec::F64}, dw, wn);
  }
  if (rout) copy(ctx, VPtr{rout, Prec::F64}, ro, L.opsize(L.a));
}

EvalOut energy_grad(Ctx& ctx, const mera_shape& shape, const Point& pt, const double* h3, Prec prec, Warm* warm,
                    const KrylovOpts& ko, const GradOut& out) {
  const std::vector<LayerDim> dims = layer_dims(shape);
  const int T = shape.T;
  const int chi = shape.chi;
  const LayerDim& S = dims[T];
  // operator side and element count at the scale-invariant layer (chi^3, chi^6 binary; chi^2, chi^4 ternary)
  const int64_t chi3 = S.opdim(chi), n6 = S.opsize(chi);
  const size_t eb = elem_bytes(prec);
  const double macs0 = ctx.macs;
  EvalOut res;
  MERA_CHECK((int)pt.u.size() == T + 1 && (int)pt.w.size() == T + 1, MERA_EINVAL, "need T+1 tensors u and w");
  MERA_CHECK((int)out.Du.size() == T + 1 && (int)out.Dw.size() == T + 1, MERA_EINVAL, "need T+1 outputs");

  // tensors in contraction precision
  std::vector<LayerTensors> lt(T + 1);
  for (int t = 0; t <= T; ++t) {
    const int64_t a2 = (int64_t)dims[t].a * dims[t].a;
    if (prec == Prec::F64) {
      lt[t] = {(void*)pt.u[t], (void*)pt.w[t]};
    } else {
      const int64_t wn = dims[t].wrows() * dims[t].b;
      lt[t].u = ctx.buf("shadow.u" + std::to_string(t), a2 * a2 * 4);
      lt[t].w = ctx.buf("shadow.w" + std::to_string(t), wn * 4);
      copy(ctx, VPtr{lt[t].u, prec}, VPtr{(void*)pt.u[t], Prec::F64}, a2 * a2);
      copy(ctx, VPtr{lt[t].w, prec}, VPtr{(void*)pt.w[t], Prec::F64}, wn);
    }
  }

  // ascend the Hamiltonian through the transition layers
  std::vector<VPtr> hs(T + 1);
  hs[0] = VPtr{ctx.buf("hs0", S.opsize(shape.d) * eb), prec};
  copy(ctx, hs[0], VPtr{(void*)h3, Prec::F64}, S.opsize(shape.d));
  // binary transition layers keep their forward activations for their derivatives when they fit the limit
  const bool cache = activation_cache_bytes(dims, eb) > 0 && activation_cache_bytes(dims, eb) <= ctx.inter_limit;
  std::vector<Activations> acts(T);
  if (cache)
    for (int t = 0; t < T; ++t) {
      const auto n = activation_elems(dims[t]);
      for (int s = 0; s < 2; ++s)
        for (int j = 0; j < 4; ++j)
          acts[t].F[s][j] = ctx.buf("act" + std::to_string(t) + "." + std::to_string(s) + "." + std::to_string(j),
                                    (size_t)n[j] * eb);
    }
  for (int t = 0; t < T; ++t) {
    hs[t + 1] = VPtr{ctx.buf("hs" + std::to_string(t + 1), S.opsize(dims[t].b) * eb), prec};
    if (cache) ascend_fwd(ctx, dims[t], lt[t], hs[t], hs[t + 1], prec, acts[t]);
    else ascend_raw(ctx, dims[t], lt[t], hs[t], hs[t + 1], prec);
  }

  // Extrapolated warm starts: with the solutions x1, x2 of the last two evaluations (at points P1, P2), both solves
  // start from x1 + t (x1 - x2), t the component of this evaluation's step P - P1 along the previous step P1 - P2
  // (a first-order prediction along the line the optimiser moves on; within a line search the points are
  // collinear). The tensors of the last two points are kept flattened in the warm-start object.
  double theta = 0.0;
  bool extrap = false;
  if (warm && ko.extrapolate) {
    int64_t ne = 0;
    for (int t = 0; t <= T; ++t) ne += (int64_t)dims[t].a * dims[t].a * dims[t].a * dims[t].a + dims[t].wrows() * dims[t].b;
    if (warm->pt_elems != ne || warm->chi != chi) {
      warm->npts = 0;
      warm->has_prev = false;
      warm->pt_elems = ne;
    }
    warm->pts[0].ensure(ne * 8);
    warm->pts[1].ensure(ne * 8);
    double* cur = static_cast<double*>(ctx.buf("warm.cur", ne * 8));
    int64_t o = 0;
    for (int t = 0; t <= T; ++t) {
      const int64_t nu = (int64_t)dims[t].a * dims[t].a * dims[t].a * dims[t].a, nw = dims[t].wrows() * dims[t].b;
      copy(ctx, VPtr{cur + o, Prec::F64}, VPtr{(void*)pt.u[t], Prec::F64}, nu);
      copy(ctx, VPtr{cur + o + nu, Prec::F64}, VPtr{(void*)pt.w[t], Prec::F64}, nw);
      o += nu + nw;
    }
    if (warm->npts >= 2 && warm->has_prev && warm->has_rho && warm->has_ht) {
      double* d1 = static_cast<double*>(ctx.buf("warm.d1", ne * 8));
      double* d0 = static_cast<double*>(ctx.buf("warm.d0", ne * 8));
      const VPtr p1{warm->pts[0].ptr, Prec::F64}, p2{warm->pts[1].ptr, Prec::F64};
      copy(ctx, VPtr{d1, Prec::F64}, VPtr{cur, Prec::F64}, ne);
      axpby(ctx, -1.0, p1, 1.0, VPtr{d1, Prec::F64}, ne);
      copy(ctx, VPtr{d0, Prec::F64}, p1, ne);
      axpby(ctx, -1.0, p2, 1.0, VPtr{d0, Prec::F64}, ne);
      const double den = dot(ctx, VPtr{d0, Prec::F64}, VPtr{d0, Prec::F64}, ne);
      if (den > 0.0 && std::isfinite(den)) {
        theta = dot(ctx, VPtr{d1, Prec::F64}, VPtr{d0, Prec::F64}, ne) / den;
        theta = std::max(-1.0, std::min(1.0, theta));
        extrap = std::isfinite(theta) && theta != 0.0;
      }
    }
  }

  const double tol = ko.tol > 0 ? ko.tol : (prec == Prec::F64 ? 1e-13 : 1e-7);
  const int kdim = ko.dim > 0 ? ko.dim : default_krylov_dim((size_t)n6 * eb);
  const int kres = ko.max_restarts > 0 ? ko.max_restarts : 200;

  // scale-invariant density matrix: x - D(x) + Tr[x] sigma = sigma, sigma = warm start with unit trace
  VPtr rho{ctx.buf("rho_s", n6 * eb), prec};
  VPtr sigma{ctx.buf("sigma", n6 * eb), prec};
  VPtr tmp{ctx.buf("ktmp", n6 * eb), prec};
  if (warm && warm->has_rho && warm->chi == chi) {
    copy(ctx, rho, VPtr{warm->rho.ptr, Prec::F64}, n6);
    if (extrap) {
      axpby(ctx, theta, VPtr{warm->rho.ptr, Prec::F64}, 1.0, rho, n6);
      axpby(ctx, -theta, VPtr{warm->rho_prev.ptr, Prec::F64}, 1.0, rho, n6);
    }
    double tr = trace(ctx, rho, chi3);
    scal(ctx, 1.0 / tr, rho, n6);
  } else {
    fill(ctx, rho, n6, 0.0);
    add_diag(ctx, rho, chi3, 1.0 / (double)chi3);
  }
  copy(ctx, sigma, rho, n6);
  double* opsc = static_cast<double*>(ctx.buf("krylov.opscalar", sizeof(double)));
  auto op_rho = [&](VPtr in, VPtr o) {
    descend_raw(ctx, S, lt[T], in, o, prec);
    axpby(ctx, 1.0, in, -1.0, o, n6);
    trace_dev(ctx, in, chi3, opsc);
    axpby_dev(ctx, opsc, 1.0, sigma, 1.0, o, n6);
  };
  KStat kr = gmres(ctx, op_rho, sigma, rho, n6, kdim, tol, kres, prec, "fixed-point");
  MERA_CHECK(kr.converged, MERA_ENOCONV,
             "fixed-point solve did not converge (residual " + std::to_string(kr.res) + ")");
  symmetrize(ctx, rho, chi3);
  {
    double tr = trace(ctx, rho, chi3);
    MERA_CHECK(std::isfinite(tr) && tr != 0.0, MERA_ENONFINITE, "bad trace of the fixed point");
    scal(ctx, 1.0 / tr, rho, n6);
  }
  res.app_rho = kr.apps;
  res.res_rho = kr.res;

  const double e = dot(ctx, hs[T], rho, n6);
  MERA_CHECK(std::isfinite(e), MERA_ENONFINITE, "non-finite energy");
  res.energy = e;

  // h~: x - A(x) + Tr[x rho] 1 = h_T - e 1
  VPtr hp{ctx.buf("hprime", n6 * eb), prec};
  VPtr ht{ctx.buf("htilde", n6 * eb), prec};
  copy(ctx, hp, hs[T], n6);
  add_diag(ctx, hp, chi3, -e);
  if (warm && warm->has_ht && warm->chi == chi) {
    copy(ctx, ht, VPtr{warm->ht.ptr, Prec::F64}, n6);
    if (extrap) {
      axpby(ctx, theta, VPtr{warm->ht.ptr, Prec::F64}, 1.0, ht, n6);
      axpby(ctx, -theta, VPtr{warm->ht_prev.ptr, Prec::F64}, 1.0, ht, n6);
    }
  } else {
    copy(ctx, ht, hp, n6);
  }
  auto op_ht = [&](VPtr in, VPtr o) {
    ascend_raw(ctx, S, lt[T], in, o, prec);
    axpby(ctx, 1.0, in, -1.0, o, n6);
    dot_dev(ctx, in, rho, n6, opsc);
    add_diag_dev(ctx, o, chi3, opsc, 1.0);
  };
  KStat kh = gmres(ctx, op_ht, hp, ht, n6, kdim, tol, kres, prec, "h~");
  MERA_CHECK(kh.converged, MERA_ENOCONV, "h~ solve did not converge (residual " + std::to_string(kh.res) + ")");
  symmetrize(ctx, ht, chi3);
  add_diag(ctx, ht, chi3, -dot(ctx, ht, rho, n6));  // gauge Tr[h~ rho] = 0
  res.app_ht = kh.apps;
  res.res_ht = kh.res;

  if (warm) {
    if (ko.extrapolate && warm->has_rho && warm->has_ht && warm->chi == chi) {
      // the current solutions become the previous ones
      warm->rho_prev.ensure(n6 * 8);
      warm->ht_prev.ensure(n6 * 8);
      std::swap(warm->rho, warm->rho_prev);
      std::swap(warm->ht, warm->ht_prev);
      warm->has_prev = true;
    }
    warm->chi = chi;
    warm->rho.ensure(n6 * 8);
    warm->ht.ensure(n6 * 8);
    copy(ctx, VPtr{warm->rho.ptr, Prec::F64}, rho, n6);
    copy(ctx, VPtr{warm->ht.ptr, Prec::F64}, ht, n6);
    warm->has_rho = warm->has_ht = true;
    if (ko.extrapolate) {
      // this point joins the history only with its solutions, so points and solutions stay paired even when an
      // evaluation fails before this
      std::swap(warm->pts[0], warm->pts[1]);
      copy(ctx, VPtr{warm->pts[0].ptr, Prec::F64}, VPtr{ctx.buf("warm.cur", 0), Prec::F64}, warm->pt_elems);
      warm->npts = std::min(2, warm->npts + 1);
    }
  }

  // gradients, top down; rl[t] = density matrix at the top of layer t (rl[T] = rho_s)
  std::vector<VPtr> rl(T + 1);
  rl[T] = rho;
  for (int t = T; t >= 0; --t) {
    const LayerDim& L = dims[t];
    const int64_t a2 = (int64_t)L.a * L.a;
    VPtr Du, Dw;
    if (prec == Prec::F64) {
      Du = VPtr{out.Du[t], prec};
      Dw = VPtr{out.Dw[t], prec};
    } else {
      Du = VPtr{ctx.buf("Dacc.u", a2 * a2 * 4), prec};
      Dw = VPtr{ctx.buf("Dacc.w", L.wrows() * L.b * 4), prec};
    }
    const VPtr hin = (t == T) ? ht : hs[t];
    const VPtr rtop = (t == T) ? rho : rl[t + 1];
    // the descended matrix is the top of layer t-1; it is not needed below layer 0 or for the
    // scale-invariant layer, whose bottom is rho_s itself
    const bool keep = (t >= 1 && t < T);
    VPtr rdown{ctx.buf(keep ? "rl" + std::to_string(t) : std::string("rl.discard"), L.opsize(L.a) * eb), prec};
    if (cache && t < T) layer_grad_rev(ctx, L, lt[t], rtop, Du, Dw, rdown, prec, acts[t]);
    else layer_grad(ctx, L, lt[t], hin, rtop, Du, Dw, rdown, prec);
    if (keep) rl[t] = rdown;
    if (prec != Prec::F64) {
      copy(ctx, VPtr{out.Du[t], Prec::F64}, Du, a2 * a2);
      copy(ctx, VPtr{out.Dw[t], Prec::F64}, Dw, L.wrows() * L.b);
    }
  }

  if (!out.rho_u.empty()) {
    MERA_CHECK((int)out.rho_u.size() == T + 1 && (int)out.rho_w.size() == T + 1, MERA_EINVAL,
               "need T+1 preconditioner outputs");
    for (int t = 0; t <= T; ++t) {
      const LayerDim& L = dims[t];
      VPtr rtop = (t == T) ? rho : rl[t + 1];
      double* r2 = static_cast<double*>(ctx.buf("rdm.rho2", (size_t)L.b * L.b * L.b * L.b * 8));
      if (L.ternary) {
        // the top two-site rho itself (FP64) feeds rho_u; rho_w averages its two one-site marginals
        copy(ctx, VPtr{r2, Prec::F64}, rtop, L.opsize(L.b));
        rho_marginal_pair(ctx, VPtr{r2, Prec::F64}, L.b, out.rho_w[t]);
      } else {
        rho_marginals(ctx, rtop, L.b, out.rho_w[t], r2);
      }
      symmetrize(ctx, VPtr{out.rho_w[t], Prec::F64}, L.b);
      run_program(ctx, L.ternary ? programs().trhou : programs().rhou, legs_of(L),
                  {{"w", (void*)pt.w[t]}, {"rho2", r2}, {"rhou", out.rho_u[t]}}, Prec::F64);
      symmetrize(ctx, VPtr{out.rho_u[t], Prec::F64}, (int64_t)L.a * L.a);
    }
  }
  res.macs = ctx.macs - macs0;
  return res;
}

}  // namespace mera
