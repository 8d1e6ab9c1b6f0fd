// Composite odd-quintic filter coefficients, f_t(x) = a x + b x^3 + c x^5.
//
// Library transcription of the refined ("tilde") tables of the paper:
//   kTildeSingle — Table 1 (single-precision setting, T = 10)
//   kTildeHalf   — Table 2 (half-precision setting, T = 7)
// Per-stage stability rescale (Section 3.4): the half-precision iterate is
// multiplied by 1/1.01 after stages 1..T-1, the single-precision iterate by
// 1/1.001 after stages 1..8; the factor is folded into (a, b, c) in FP64 before
// the coefficients reach a kernel. (Rescaling after the last half-precision
// stage as well would bias sign(x) to 1/1.01 and cap the ReLU error near
// 5e-3, which the paper's reported half-precision errors rule out.)
#pragma once

namespace psd {

struct StageCoef { double a, b, c; };

constexpr StageCoef kTildeSingle[10] = {
    {8.3119043343, -23.0739115930, 16.4664144722},
    {4.1439360087, -2.9176674704, 0.5246212487},
    {4.0257813209, -2.9025002398, 0.5334261214},
    {3.5118574347, -2.5740236523, 0.5050097282},
    {2.4398158400, -1.7586675341, 0.4191290613},
    {1.9779835097, -1.3337358510, 0.3772169049},
    {1.9559726949, -1.3091355170, 0.3746734515},
    {1.9282822454, -1.2823649693, 0.3704626545},
    {1.9220135179, -1.2812524618, 0.3707011753},
    {1.8942192942, -1.2613293407, 0.3676616051},
};

constexpr StageCoef kTildeHalf[7] = {
    {8.2885332412, -22.5927099246, 15.8201383114},
    {4.1666196466, -2.9679004036, 0.5307623217},
    {4.0611848147, -2.9698947955, 0.5492133813},
    {3.6678301399, -2.7561018955, 0.5421513305},
    {2.7632556383, -2.0607754898, 0.4695405857},
    {2.0527445797, -1.4345145882, 0.4070669182},
    {1.8804816691, -1.2583997294, 0.3779501813},
};

// Newton-Schulz baseline compared against in Section 4.1: the cubic sign
// iteration x <- (3 x - x^3) / 2, 10 steps in half precision and 15 in single
// precision (21 and 31 products with the final one), without stage rescale.
constexpr StageCoef kNewtonSchulz = {1.5, -0.5, 0.0};
constexpr int kNewtonSchulzHalf = 10;
// Quintic Newton-Schulz step (15 x - 10 x^3 + 3 x^5) / 8 (the last two stages
// of Table 1's Stage-I column): the extra stages of adaptive depth.
constexpr StageCoef kNewtonSchulzQuintic = {15.0 / 8.0, -10.0 / 8.0, 3.0 / 8.0};
constexpr int kNewtonSchulzSingle = 15;

// Number of stages followed by the 1/1.001 (single) or 1/1.01 (half) rescale.
constexpr int kSingleRescaled = 8;
constexpr double kSingleRescale = 1.0 / 1.001;
constexpr int kHalfRescaled = 6;
constexpr double kHalfRescale = 1.0 / 1.01;

}  // namespace psd
