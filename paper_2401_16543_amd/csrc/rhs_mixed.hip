// Split-precision KFVM-WENO right-hand side for gfx950 (matrix cores).
//
// The weight-apply and smoothness-indicator contractions run on
// v_mfma_f32_32x32x16_{f16,bf16}: each operand x is split into hi = half(x) and
// lo = half(x - hi), and A.B ~ A_hi B_hi + A_hi B_lo + A_lo B_hi is accumulated
// in float32.  The increments fed to the matrix cores are formed in float64;
// the smoothness-indicator sums of squares and the blend sums take the float32
// accumulator values; the nonlinear weights and their normalisation are float64
// (eps = 1e-40 is far below the float32 range), and so are the positivity
// limiter, the Riemann solver and the Runge-Kutta update.
//
// Contraction layout (one wave = 32 cells, both half-waves on the same cells):
//   B (K x N): the increments delta_h = W_h - W_c of one reconstruction variable
//      over S0 less its centre (whose increment is zero; K padded to 16), for
//      the wave's 32 cells (N).  Because the point rows of every table sum to
//      one and the derivative rows to zero, point values are W_c + R.delta and
//      derivatives R.delta exactly; the increments are small on smooth data, so
//      the split keeps ~22 significant bits of them.  They are scaled per cell
//      by a power of two to [2^13, 2^14).
//   A (M x K): every stencil's table embedded in S0 columns (zeros outside the
//      stencil), rows interleaved as target * 8 + stencil, weights scaled by 2^SW.
//      In the 32 x 32 accumulator layout a lane then holds, for each of four
//      targets per tile, the values of four stencils (stencils 0-3 in the lower
//      half-wave, 4-7 in the upper): the smoothness indicators and the blend are
//      lane-local partial sums plus one exchange between the half-waves.
//   A second table holds only the S0 face-point rows (targets as rows): a wave
//   whose 32 cells the gate marks as smooth for a variable uses it alone.
// The tables sit in LDS; for 3D R = 3 they are too large and stream through an
// LDS window (k_recon_mixed_stream).
// The kernel writes the blended increments w_s - W_c as float32 (half the bytes
// of the float64 path; the value is a float32 matrix-core sum to begin with),
// and the limiter's two factors, found from running bounds of the stored
// increments; the face-flux kernel rebuilds u_s = U_c + theta Phi^-1 (w_s - W_c).
#include "device_common.hpp"

namespace kfvm {
namespace {
using namespace dev;

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 bh8 __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));

constexpr int SB = 13;   // per-cell increment scale: max |delta| * 2^(SB - e) in [2^13, 2^14)
// Least exponent e of that scale, so that 2^(SB - e) stays finite: increments
// ahead of a wave front decay to float64 denormals (seen: 6e-314), whose scale
// would overflow.  Below 2^e_min the increments are scaled by less than the
// nominal factor; they are far under float32's range anyway.
constexpr int E_MIN_D = -1000;      // float64 scaling
constexpr int E_MIN_F = SB - 127;   // float32 scaling (2^127 is the largest finite power)
constexpr double FLAT_REL = 0x1p-40;   // gate: increments below this fraction of the scale are flat

// 3D tiles are 8 x 8 x 8 here (8 x 8 x 4 for R = 3): the threads of a block
// (two lanes per cell) share one copy of the operand tables in LDS
template <int D, int R>
using MCfg = Cfg<D, R, (D == 3 ? (R == 2 ? 8 : 4) : 1)>;

template <int D, int R>
struct MixCfg {
    using S = Stencil<D, R>;
    static constexpr int NK = S::N0 - 1;                        // S0 without its centre
    static constexpr int KS = (NK + 15) / 16;                   // k-steps of 16
    static constexpr int NTF = (S::NROWS * 8 + 31) / 32;        // interleaved tiles
    static constexpr int TP_END = (S::NPTS * 8 + 31) / 32;      // tiles holding point rows
    static constexpr int TD_BEGIN = (S::NPTS * 8) / 32;         // first tile holding derivative rows
    static constexpr int NTL = (S::NPTS + 31) / 32;             // S0-only tiles
    static constexpr int A_FULL = NTF * KS * 2 * 64;            // 16-byte operand slots
    static constexpr int A_LIN = NTL * KS * 2 * 64;
    static constexpr int NT = 2 * MCfg<D, R>::NT;                // two lanes per cell
};

// the 3D R = 3 operand tables exceed LDS and are streamed through it
constexpr bool streamed_tables(int dim, int R) { return dim == 3 && R == 3; }

// ---------------------------------------------------- half-wave exchange ---
// v_permlane32_swap trades the upper half of its first register with the lower
// half of its second; with both set to x it returns {x_lo, x_lo} and
// {x_hi, x_hi} (x_lo: the value of lanes 0-31, x_hi: lanes 32-63).
__device__ __forceinline__ void halves(uint32_t x, uint32_t &lo, uint32_t &hi)
{
    const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    lo = r[0];
    hi = r[1];
}
__device__ __forceinline__ void halves(float x, float &lo, float &hi)
{
    uint32_t a, b;
    halves(__builtin_bit_cast(uint32_t, x), a, b);
    lo = __builtin_bit_cast(float, a);
    hi = __builtin_bit_cast(float, b);
}
__device__ __forceinline__ void halves(double x, double &lo, double &hi)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    uint32_t l0, h0, l1, h1;
    halves((uint32_t)u, l0, h0);
    halves((uint32_t)(u >> 32), l1, h1);
    lo = __builtin_bit_cast(double, (uint64_t)l0 | (uint64_t)l1 << 32);
    hi = __builtin_bit_cast(double, (uint64_t)h0 | (uint64_t)h1 << 32);
}
template <typename T>
__device__ __forceinline__ T pair_sum(T x) { T a, b; halves(x, a, b); return a + b; }
template <typename T>
__device__ __forceinline__ T pair_max(T x) { T a, b; halves(x, a, b); return a > b ? a : b; }
template <typename T>
__device__ __forceinline__ T pair_min(T x) { T a, b; halves(x, a, b); return a < b ? a : b; }
template <typename T>
__device__ __forceinline__ T lower_half(T x) { T a, b; halves(x, a, b); return a; }
template <typename T>
__device__ __forceinline__ T partner(T x, int hf) { T a, b; halves(x, a, b); return hf ? a : b; }

// element at byte offset uoff + off of a kernel-argument array: uoff is
// wave-uniform (read from the first lane, so it lives in scalar registers) and
// off a per-lane offset below 2^32, which gives the scalar-base + 32-bit
// lane-offset addressing form
template <typename T>
__device__ __forceinline__ T &at4(T *base, long uoff, uint32_t off)
{
    // (the builtin returns a signed int: widen each half through uint32_t)
    const uint64_t u = (uint64_t)uoff;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    const long us = (long)((uint64_t)lo | (uint64_t)hi << 32);
    return *reinterpret_cast<T *>(reinterpret_cast<char *>(const_cast<std::remove_const_t<T> *>(base)) + us + off);
}

template <bool BF>
__device__ __forceinline__ f16v mfma(uint4 a, uint4 b, f16v c)
{
    if constexpr (BF)
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bh8, a), __builtin_bit_cast(bh8, b), c, 0, 0,
                                                       0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(h8, a), __builtin_bit_cast(h8, b), c, 0, 0, 0);
}

// hi/lo split of two scaled increments into packed 16-bit pairs: hi rounds to
// nearest, the residual y - hi is exact in float32 and is rounded the same way,
// so hi + lo keeps ~22 (fp16) or ~16 (bf16) significant bits of y.  Pairs go
// through the packed float32 -> 16-bit conversions.
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
typedef __bf16 b2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));

template <bool BF>
__device__ __forceinline__ void split_pair(float ya, float yb, uint32_t &hi, uint32_t &lo)
{
    using T2 = std::conditional_t<BF, b2v, h2v>;
    const f2v y = {ya, yb};
    const T2 h = __builtin_convertvector(y, T2);
    hi = __builtin_bit_cast(uint32_t, h);
    if constexpr (BF) {
        const f2v hf = __builtin_convertvector(h, f2v);
        const f2v r = {ya - hf.x, yb - hf.y};
        lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, T2));
    } else {
        // the mixed-precision FMA reads each FP16 half of hi as an operand and
        // rounds the float32 result y - hi (exact) once to FP16: the same
        // residual as widening hi, subtracting and converting, in one
        // instruction per value instead of two and a half.  The compiler does
        // not see a VALU write in the asm, so the asm itself ends with the two
        // wait states a matrix-core read of the result may need.
        asm("v_fma_mixlo_f16 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]\n\t"
            "v_fma_mixhi_f16 %0, -%1, 1.0, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]\n\t"
            "s_nop 1"
            : "=&v"(lo)
            : "v"(hi), "v"(ya), "v"(yb));
    }
}

// increment of variable K at contraction slots kA (lower half-wave) and kB
// (upper), zero past the last slot; LDS offsets fold into immediates
template <int D, int R, int K>
__device__ __forceinline__ double slot_increment(const double (*tile)[MCfg<D, R>::HN], int lc, int hf, int kA, int kB,
                                                 const PhiRows<D> &ph, double Wc)
{
    using C = MCfg<D, R>;
    constexpr int NK = MixCfg<D, R>::NK;
    const int hA = slot_point<D, R>(kA < NK ? kA : 0), hB = slot_point<D, R>(kB < NK ? kB : 0);
    const int oA = kA < NK ? C::st.off[hA][0] + C::HX * (C::st.off[hA][1] + C::HY * C::st.off[hA][2]) : 0;
    const int oB = kB < NK ? C::st.off[hB][0] + C::HX * (C::st.off[hB][1] + C::HY * C::st.off[hB][2]) : 0;
    const bool valid = hf ? (kB < NK) : (kA < NK);
    const int o = lc + (hf ? oB : oA);
    const double w = w_component<D, K, C::HN>(tile, o, ph);
    return valid ? w - Wc : 0.0;
}

// ------------------------------------------------------------ learned gate ---
// The troubled-cell network (n_in -> 32 -> 32 -> 1, GELU) evaluated for the
// wave's 32 cells on BF16 matrix cores with float32 accumulation.  Its inputs
// are the increments W_h - W_c of this variable divided by 2^ex, the power of
// two just above their largest magnitude: in 3D the S0 increments the
// reconstruction already holds (its float32 operands are those inputs times
// 2^(SB+1); W1 carries the factor 2^-(SB+1), an exact exponent shift), in 2D
// the 5 x 5 window around the cell.  The S0 centre, always zero, has no slot.
// Operand slots (per lane, 8 BF16 values): W1 [KSG][64], W2 [2][64]; vec holds
// b1 [32], b2 [32], w3 [32], b3.
template <int D>
struct GateShape {
    static constexpr int NIN = D == 2 ? 25 : 33;
    static constexpr int KSG = 2;                 // 25 window values / 32 S0 slots
    static constexpr int SLOTS = (KSG + 2) * 64;
};

__device__ __forceinline__ f16v mfma_bf16(uint4 a, uint4 b, f16v c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bh8, a), __builtin_bit_cast(bh8, b), c, 0, 0, 0);
}

// two floats to a BF16 pair (a in the low half), rounded to nearest even, by
// one packed conversion
__device__ __forceinline__ uint32_t pack_bf16(float a, float b)
{
    const f2v v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, b2v));
}

// 16 accumulator registers from vec[base + unit]: register j holds unit
// 8 (j / 4) + 4 hf + j % 4 of a 32 x 32 accumulator
__device__ __forceinline__ f16v unit_regs(const float *vec, int hf)
{
    f16v a;
#pragma unroll
    for (int gq = 0; gq < 4; ++gq) {
        const float4 b = *reinterpret_cast<const float4 *>(vec + 8 * gq + 4 * hf);
        a[4 * gq + 0] = b.x;
        a[4 * gq + 1] = b.y;
        a[4 * gq + 2] = b.z;
        a[4 * gq + 3] = b.w;
    }
    return a;
}

// GELU of the inference by chords: bin k of width 1/64 centred on
// z = (k - 384) / 64 (k = 0 .. 767, so the bins tile [-6 - 1/128, 6 - 1/128))
// holds (a_k, b_k), the line through gelu_f at the bin's ends; beyond the first
// and last bins their chords continue (GELU is 0 or z there to 1e-8).  The
// chords are within 2.5e-5 of gelu_f, far below the BF16 rounding of the hidden
// layer, and cost one LDS read and four plain VALU operations against the
// exponential and reciprocal of gelu_f, which the VALU-bound gated
// reconstruction feels.  The table sits in LDS after the gate's vector
// parameters (GVEC_TAB floats on).
constexpr int GELU_NB = 768;
constexpr int GVEC_TAB = 104;                          // after b1, b2, w3, b3 (97 floats), 16-byte aligned
constexpr int GVEC_SIZE = GVEC_TAB + 2 * GELU_NB;
// 1.5 * 2^23: the floats of [2^23, 2^24) are the integers, so adding it rounds
// to the nearest integer and leaves that integer in the low mantissa bits
constexpr float GELU_MAGIC = 12582912.f;

__device__ __forceinline__ void gelu_table_fill(float *gvec, int tid, int nt)
{
    float2 *tab = reinterpret_cast<float2 *>(gvec + GVEC_TAB);
    for (int k = tid; k < GELU_NB; k += nt) {
        const float z0 = -6.f + ((float)k - 0.5f) * (1.f / 64.f), z1 = z0 + 1.f / 64.f;
        const float g0 = gelu_f(z0), g1 = gelu_f(z1);
        const float b = (g1 - g0) * 64.f;
        tab[k] = make_float2(g0 - b * z0, b);
    }
}

__device__ __forceinline__ float gelu_tab(float z, const float *gvec)
{
    const float2 *tab = reinterpret_cast<const float2 *>(gvec + GVEC_TAB);
    // bin k = the integer nearest 64 z + 384, formed by the magic add and
    // clamped in float to [0, 767] (fmaxf of NaN gives the lower end, so any z
    // stays in range); its bits less the magic's are k
    const float t = fminf(fmaxf(fmaf(z, 64.f, 384.f + GELU_MAGIC), GELU_MAGIC), GELU_MAGIC + (float)(GELU_NB - 1));
    const uint32_t k = __float_as_uint(t) - __float_as_uint(GELU_MAGIC);
    const float2 c = tab[k];
    return fmaf(c.y, z, c.x);
}

// logit of this lane's cell (identical in both half-waves); xb: the lane's BF16
// input operands.  Both layers start their accumulators from the biases.
template <int D>
__device__ __forceinline__ float gate_forward(const uint4 (&xb)[GateShape<D>::KSG], int lane, const uint4 *Wg,
                                              const float *vec)
{
    constexpr int KSG = GateShape<D>::KSG;
    const int hf = lane >> 5;
    f16v acc = unit_regs(vec, hf);
#pragma unroll
    for (int ks = 0; ks < KSG; ++ks) acc = mfma_bf16(Wg[ks * 64 + lane], xb[ks], acc);
    uint32_t P[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        P[p] = pack_bf16(gelu_tab(acc[2 * p], vec), gelu_tab(acc[2 * p + 1], vec));
        asm volatile("" : "+v"(P[p]));
    }
    // to the B layout (unit 16 ks + 8 hf + i): P[p] holds units
    // 8 (p / 2) + 4 hf + 2 (p % 2) and the next; one exchange of P[p] with
    // P[p + 2] leaves the first register with units 16 ks + 8 hf + {0..3} and
    // the second with 16 ks + 8 hf + {4..7} in both half-waves (ks = p / 4)
    const auto s02 = __builtin_amdgcn_permlane32_swap(P[0], P[2], false, false);
    const auto s13 = __builtin_amdgcn_permlane32_swap(P[1], P[3], false, false);
    const auto s46 = __builtin_amdgcn_permlane32_swap(P[4], P[6], false, false);
    const auto s57 = __builtin_amdgcn_permlane32_swap(P[5], P[7], false, false);
    const uint4 b0 = make_uint4(s02[0], s13[0], s02[1], s13[1]);
    const uint4 b1 = make_uint4(s46[0], s57[0], s46[1], s57[1]);
    f16v acc2 = unit_regs(vec + 32, hf);
    acc2 = mfma_bf16(Wg[(KSG + 0) * 64 + lane], b0, acc2);
    acc2 = mfma_bf16(Wg[(KSG + 1) * 64 + lane], b1, acc2);
    const f16v w3 = unit_regs(vec + 64, hf);
    float part = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) part = fmaf(w3[j], gelu_tab(acc2[j], vec), part);
    return pair_sum(part) + vec[96];
}

// Running bounds of a cell's stored face-point increments for the positivity
// limiter: least and largest density increment, least pressure-row increment,
// and the sum over the velocity rows of their largest square.  Each half-wave
// bounds the points it stores; settle_bounds merges the two.
struct IncBounds {
    float rlo = INFINITY, rhi = -INFINITY, plo = INFINITY, v2 = 0.f;
};

template <int D, int K>
__device__ __forceinline__ void note_increment(IncBounds &b, float x, float &v2k)
{
    if constexpr (K == 0) {
        b.rlo = fminf(b.rlo, x);
        b.rhi = fmaxf(b.rhi, x);
    } else if constexpr (K == D + 1) {
        b.plo = fminf(b.plo, x);
    } else {
        v2k = fmaxf(v2k, x * x);
    }
}

// Face point tau of a cell is stored, and enters the limiter's bounds, in the
// half-wave hf = bit 2 of tau: in the S0-only layout the accumulator holds
// point T0 in the lower half-wave and T0 + 4 in the upper (T0 with bit 2
// clear), so each lane keeps what it computed; the blended layout takes the
// point tiles in pairs (t even: bit 2 clear, t + 1: set) and one exchange per
// target gives each half-wave the sums of its own tile.  The bounds are then
// per lane, and settle_bounds merges the two halves of a cell.
__device__ __forceinline__ int owner_half(int tau) { return (tau >> 2) & 1; }

__device__ __forceinline__ void settle_bounds(IncBounds &b)
{
    b.rlo = pair_min(b.rlo);
    b.rhi = pair_max(b.rhi);
    b.plo = pair_min(b.plo);
}

// store the float32 increments of variable K at this lane's group of four
// points, tau_lo .. tau_lo + 3 in the lower half-wave and tau_lo + 4 .. tau_lo + 7
// in the upper (tau_lo a multiple of 8), as one vector: the lane offset lo16
// holds the cell's 16-byte column plus, in the upper half, the 16 ncell bytes
// between the two groups (inc_index)
template <int NV, int K>
__device__ __forceinline__ void store_group(float *inc, int tau_lo, long ncell, uint32_t lo16, float4 val)
{
    at4(reinterpret_cast<float4 *>(inc), 4 * inc_index(tau_lo, K, NV, ncell), lo16) = val;
}

// the blended value of the lane's own tile of a pair from its partial sums p0
// (tile t) and p1 (tile t + 1): the lower half adds the upper half's p0, the
// upper half the lower half's p1 (in the order lower + upper)
__device__ __forceinline__ float pair_blend(float p0, float p1, int hf)
{
    float lo, hi;
    halves(hf ? p0 : p1, lo, hi);
    return hf ? lo + p1 : p0 + hi;
}

template <int D, int R, int K, bool BF, bool GATE>
__device__ __forceinline__ void mixed_var(const double (*tile)[MCfg<D, R>::HN], int lc, int lane, const uint4 *As,
                                          const uint4 *Al, const PhiRows<D> &ph, int wbits,
                                          float *__restrict__ inc, uint32_t co, long ncell, bool active, int sw,
                                          const uint4 *Wg, const float *gvec, float thr, uint8_t *__restrict__ fl_out,
                                          const float (&wsc)[3], IncBounds &bnd)
{
    using C = MCfg<D, R>;
    using M = MixCfg<D, R>;
    using S = typename C::S;
    constexpr int NV = C::NV, NST = S::NST, NPTS = S::NPTS, NROWS = S::NROWS, KS = M::KS;
    const int hf = lane >> 5;
    const double Wc = w_component<D, K, C::HN>(tile, lc, ph);

    // increments over this lane's slots 16 ks + 8 hf + i; the next k-step's
    // LDS index waits for this one's values (empty asm), so at most one
    // k-step's reads are in flight
    double dl[KS][8];
    double amax = 0.0;
    int lcc = lc;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            dl[ks][i] = slot_increment<D, R, K>(tile, lcc, hf, 16 * ks + i, 16 * ks + 8 + i, ph, Wc);
            amax = fmax(amax, fabs(dl[ks][i]));
        }
        asm volatile("" : "+v"(lcc) : "v"(dl[ks][7]));
    }
    amax = pair_max(amax);
    int ex = 0;
    if (amax > 0.0) frexp(amax, &ex);          // amax in [2^(ex-1), 2^ex)
    const int e = max(ex - 1, E_MIN_D);
    const double sc = ldexp(1.0, SB - e);
    const int ue = e - SB - sw;                    // accumulator units: value = acc * 2^ue
    // scaled increments in float32 (kept as such: otherwise the two roundings
    // below fold into one software float64 -> half conversion)
    float ys[KS][8];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            ys[ks][i] = (float)(dl[ks][i] * sc);
            asm volatile("" : "+v"(ys[ks][i]));
        }
    uint4 bh[KS], bl[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        uint32_t h[4], l[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) split_pair<BF>(ys[ks][2 * i], ys[ks][2 * i + 1], h[i], l[i]);
        bh[ks] = make_uint4(h[0], h[1], h[2], h[3]);
        bl[ks] = make_uint4(l[0], l[1], l[2], l[3]);
    }

    bool use_weno = wbits < 0 || ((wbits >> K) & 1) != 0;
    if constexpr (GATE) {
        constexpr int KSG = GateShape<D>::KSG;
        uint4 xb[KSG];
        if constexpr (D == 3) {
            static_assert(KSG == KS, "the 3D gate reads the contraction slots");
#pragma unroll
            for (int ks = 0; ks < KSG; ++ks)
                xb[ks] = make_uint4(pack_bf16(ys[ks][0], ys[ks][1]), pack_bf16(ys[ks][2], ys[ks][3]),
                                    pack_bf16(ys[ks][4], ys[ks][5]), pack_bf16(ys[ks][6], ys[ks][7]));
        } else {
            // 5 x 5 window, slot w = 16 ks + 8 hf + i <-> offset (w / 5 - 2, w % 5 - 2)
            double gw[KSG][8], gmax = 0.0;
            int lg = lc;
#pragma unroll
            for (int ks = 0; ks < KSG; ++ks) {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int wA = 16 * ks + i, wB = 16 * ks + 8 + i;
                    const int oA = wA < 25 ? (wA / 5 - 2) + C::HX * (wA % 5 - 2) : 0;
                    const int oB = wB < 25 ? (wB / 5 - 2) + C::HX * (wB % 5 - 2) : 0;
                    const bool okw = hf ? (wB < 25) : (wA < 25);
                    const double w = w_component<D, K, C::HN>(tile, lg + (hf ? oB : oA), ph);
                    gw[ks][i] = okw ? w - Wc : 0.0;
                    gmax = fmax(gmax, fabs(gw[ks][i]));
                }
                asm volatile("" : "+v"(lg) : "v"(gw[ks][7]));
            }
            gmax = pair_max(gmax);
            int gex = 0;
            if (gmax > 0.0) frexp(gmax, &gex);
            const double gs = ldexp(1.0, -max(gex, E_MIN_D));
#pragma unroll
            for (int ks = 0; ks < KSG; ++ks) {
                float gx[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) gx[i] = (float)(gw[ks][i] * gs);
                xb[ks] = make_uint4(pack_bf16(gx[0], gx[1]), pack_bf16(gx[2], gx[3]), pack_bf16(gx[4], gx[5]),
                                    pack_bf16(gx[6], gx[7]));
            }
        }
        const float logit = gate_forward<D>(xb, lane, Wg, gvec);
        // increments at rounding level (below 2^-40 of the variable's scale:
        // density, sound speed or pressure) leave every stencil at W_c and
        // WENO-AO at the linear value to rounding: smooth whatever the network
        // says (its normalised inputs would be rounding noise)
        use_weno = logit > thr && amax > (double)wsc[K == 0 ? 0 : (K <= D ? 1 : 2)];
        if (active && hf == 0) at4(fl_out, (long)K * ncell, co) = use_weno ? 1 : 0;
    }
    const uint32_t lo16 = co * 16u + (uint32_t)hf * (uint32_t)(16 * ncell);
    float v2k = 0.f;
    if (__any(use_weno && active)) {
        // smoothness indicators: float32 sums of squares over this lane's four
        // stencils (q = 4 hf + i), in accumulator units squared
        float bp[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = M::TD_BEGIN; t < M::NTF; ++t) {
            f16v acc = {};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const uint4 ah = As[((t * KS + ks) * 2 + 0) * 64 + lane];
                const uint4 al = As[((t * KS + ks) * 2 + 1) * 64 + lane];
                acc = mfma<BF>(ah, bh[ks], acc);
                acc = mfma<BF>(ah, bl[ks], acc);
                acc = mfma<BF>(al, bh[ks], acc);
            }
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int tau = 4 * t + j / 4;
                if (tau >= NPTS && tau < NROWS) bp[j % 4] += acc[j] * acc[j];
            }
        }
        // nonlinear weights (eq. nlinWts) of this lane's four stencils in FP64;
        // the normalising sum and omega_0 come from the partner half-wave
        double om[4], part = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int q = 4 * hf + i;
            const double beta = ldexp((double)bp[i], 2 * ue);
            om[i] = q < NST ? lin_w<D>(q) * rcp64(beta * beta + EPS_WENO) : 0.0;
            part += om[i];
        }
        const double inv = rcp64(pair_sum(part));
#pragma unroll
        for (int i = 0; i < 4; ++i) om[i] *= inv;
        const double om0 = lower_half(om[0]);
        // WENO-AO coefficients (eq. wenoAOrec) of this lane's stencils, or the
        // linear S0 value for a cell the gate marks smooth
        float cm[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int q = 4 * hf + i;
            double cq = q == 0 ? om0 * inv_lin0<D>() : (q < NST ? om[i] - om0 * lin_ratio<D>(q) : 0.0);
            if (!use_weno) cq = q == 0 ? 1.0 : 0.0;
            cm[i] = (float)cq;
        }
        // blended face-point increments, point tiles in pairs
#pragma unroll
        for (int t = 0; t < M::TP_END; t += 2) {
            f16v acc0 = {}, acc1 = {};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const uint4 ah = As[((t * KS + ks) * 2 + 0) * 64 + lane];
                const uint4 al = As[((t * KS + ks) * 2 + 1) * 64 + lane];
                acc0 = mfma<BF>(ah, bh[ks], acc0);
                acc0 = mfma<BF>(ah, bl[ks], acc0);
                acc0 = mfma<BF>(al, bh[ks], acc0);
            }
            if (t + 1 < M::TP_END) {
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    const uint4 ah = As[(((t + 1) * KS + ks) * 2 + 0) * 64 + lane];
                    const uint4 al = As[(((t + 1) * KS + ks) * 2 + 1) * 64 + lane];
                    acc1 = mfma<BF>(ah, bh[ks], acc1);
                    acc1 = mfma<BF>(ah, bl[ks], acc1);
                    acc1 = mfma<BF>(al, bh[ks], acc1);
                }
            }
            float grp[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int gq = 0; gq < 4; ++gq) {
                if (4 * t + gq < NPTS) {
                    float p0 = 0.f, p1 = 0.f;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        p0 += cm[i] * acc0[4 * gq + i];
                        p1 += cm[i] * acc1[4 * gq + i];
                    }
                    grp[gq] = ldexpf(pair_blend(p0, p1, hf), ue);
                    if (4 * (t + hf) + gq < NPTS) note_increment<D, K>(bnd, grp[gq], v2k);
                }
            }
            if (active) store_group<NV, K>(inc, 4 * t, ncell, lo16, make_float4(grp[0], grp[1], grp[2], grp[3]));
        }
    } else {
        // every cell of the wave is linear for this variable: S0 face rows only
#pragma unroll
        for (int t = 0; t < M::NTL; ++t) {
            f16v acc = {};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const uint4 ah = Al[((t * KS + ks) * 2 + 0) * 64 + lane];
                const uint4 al = Al[((t * KS + ks) * 2 + 1) * 64 + lane];
                acc = mfma<BF>(ah, bh[ks], acc);
                acc = mfma<BF>(ah, bl[ks], acc);
                acc = mfma<BF>(al, bh[ks], acc);
            }
#pragma unroll
            for (int G = 0; G < 4; ++G) {
                // registers 4 G .. 4 G + 3 hold points T0 .. T0 + 3 in the lower
                // half-wave, T0 + 4 .. T0 + 7 in the upper
                const int T0 = 32 * t + 8 * G;
                if (T0 < NPTS) {
                    float grp[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        grp[i] = ldexpf(acc[4 * G + i], ue);
                        if (T0 + i + 4 < NPTS || (hf == 0 && T0 + i < NPTS)) note_increment<D, K>(bnd, grp[i], v2k);
                    }
                    if (active) store_group<NV, K>(inc, T0, ncell, lo16, make_float4(grp[0], grp[1], grp[2], grp[3]));
                }
            }
        }
    }
    if constexpr (K >= 1 && K <= D) bnd.v2 += pair_max(v2k);
}

template <int D, int R, bool BF, bool GATE, int... K>
__device__ __forceinline__ void mixed_all_vars(const double (*tile)[MCfg<D, R>::HN], int lc, int lane, const uint4 *As,
                                               const uint4 *Al, const PhiRows<D> &ph, int wbits,
                                               float *inc, uint32_t co, long ncell, bool active, int sw,
                                               const uint4 *Wg, const float *gvec, float thr, uint8_t *fl_out,
                                               const float (&wsc)[3], IncBounds &bnd,
                                               std::integer_sequence<int, K...>)
{
    ((mixed_var<D, R, K, BF, GATE>(tile, [&] { int l = lc; asm volatile("" : "+v"(l)); return l; }(), lane, As, Al,
                                   ph, wbits, inc, co, ncell, active, sw, Wg, gvec, thr, fl_out, wsc, bnd)),
     ...);
}

// Tile of conserved averages plus its R-cell halo (the ghost fill: periodic
// wrap, or the boundary conditions of non-periodic axes) into LDS; with the
// limiter on, also each tile cell's pressure (-1 where the average is not
// admissible) for the neighbourhood bounds.  In two phases: issue() puts every
// global load of the thread in flight (its tile cells sit in registers), and
// commit() writes them to LDS, so that a block's prologue waits for memory once
// rather than once per strided pass.  A tile whose halo crosses a
// non-periodic boundary fills its ghosts cell by cell in commit().
template <int D, int R, int NTHR>
struct TileLoad {
    using C = MCfg<D, R>;
    static constexpr int NV = C::NV, NIT = (C::HN + NTHR - 1) / NTHR;
    double u[NIT][NV];
    bool ghosts = false;

    __device__ __forceinline__ void issue(const double *__restrict__ U, const Geom &g, int x0, int y0, int z0)
    {
        if (!g.periodic) {
            const int o[3] = {x0, y0, z0}, h[3] = {C::HX, C::HY, C::HZ};
#pragma unroll
            for (int a = 0; a < D; ++a)
                ghosts = ghosts || (g.bc[a][0] != BC_PERIODIC && (o[a] < 0 || o[a] + h[a] > g.n[a]));
        }
        if (ghosts) return;
        // a single conditional wrap reaches every halo index once the grid is at
        // least a tile plus R wide along each axis; smaller grids take the modulo
        const bool near = g.n[0] >= C::TX + R && g.n[1] >= C::TY + R && (D == 2 || g.n[2] >= C::TZ + R);
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            // past the tile's end a thread reloads its last cell and stores nothing
            const int i = min((int)threadIdx.x + it * NTHR, C::HN - 1);
            const int hx = i % C::HX, hy = (i / C::HX) % C::HY, hz = i / (C::HX * C::HY);
            const int gx = near ? wrapi(x0 + hx, g.n[0]) : wrap_any(x0 + hx, g.n[0]);
            const int gy = near ? wrapi(y0 + hy, g.n[1]) : wrap_any(y0 + hy, g.n[1]);
            const int gz = D == 3 ? (near ? wrapi(z0 + hz, g.n[2]) : wrap_any(z0 + hz, g.n[2])) : 0;
            const long cl = gx + (long)g.n[0] * (gy + (long)g.n[1] * gz);
#pragma unroll
            for (int v = 0; v < NV; ++v) u[it][v] = U[v * g.ncell + cl];
        }
    }

    template <typename PT>
    __device__ __forceinline__ void commit(const double *__restrict__ U, const Geom &g, const Limiter &lim, int x0,
                                           int y0, int z0, double (*tile)[C::HN], PT *ptile)
    {
        const double gam = g.gamma;
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int i = (int)threadIdx.x + it * NTHR;
            if (i >= C::HN) break;
            if (ghosts) {
                const int hx = i % C::HX, hy = (i / C::HX) % C::HY, hz = i / (C::HX * C::HY);
                ghost_load<D>(U, g, x0 + hx, y0 + hy, D == 3 ? z0 + hz : 0, u[it]);
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) tile[v][i] = u[it][v];
            if (lim.on) {
                double mm = 0.0;
                bool fin = true;
#pragma unroll
                for (int v = 0; v < NV; ++v) fin = fin && isfinite(u[it][v]);
#pragma unroll
                for (int a = 0; a < D; ++a) mm += u[it][1 + a] * u[it][1 + a];
                const double p = (gam - 1.0) * (u[it][D + 1] - 0.5 * mm * rcp64(u[it][0]));
                ptile[i] = (PT)(fin && u[it][0] > 0.0 && p > 0.0 ? p : -1.0);
            }
        }
    }
};

template <int D, int R, int NTHR, typename PT>
__device__ __forceinline__ void load_tile(const double *__restrict__ U, const Geom &g, const Limiter &lim, int x0,
                                          int y0, int z0, double (*tile)[MCfg<D, R>::HN], PT *ptile)
{
    TileLoad<D, R, NTHR> tl;
    tl.issue(U, g, x0, y0, z0);
    tl.commit(U, g, lim, x0, y0, z0, tile, ptile);
}

// An operand table that every block holds in LDS, N 16-byte slots (a multiple
// of 64), straight from global memory into LDS (global_load_lds, no registers):
// wave w of NW copies rows w, w + NW, ... of 64 slots.  Complete once the
// issuing wave has waited for its vector memory counter.
template <int N, int NW>
__device__ __forceinline__ void lds_rows(const uint4 *__restrict__ src, uint4 *dst, int wave, int lane)
{
    static_assert(N % 64 == 0, "whole rows of 64 slots");
    typedef __attribute__((address_space(1))) void *gptr;
    typedef __attribute__((address_space(3))) void *lptr;
#pragma unroll
    for (int r = wave; r < N / 64; r += NW)
        __builtin_amdgcn_global_load_lds((gptr)(src + r * 64 + lane), (lptr)(dst + r * 64), 16, 0, 0);
}

// N elements of a small table, copied by NT threads in the same two phases as
// the tile: load() issues the thread's global loads (past the end it reloads
// the last element), store() writes what is in range
template <int N, int NT, typename T>
struct LdsCopy {
    static constexpr int NIT = (N + NT - 1) / NT;
    T r[NIT];
    __device__ __forceinline__ void load(const T *__restrict__ src)
    {
#pragma unroll
        for (int it = 0; it < NIT; ++it) r[it] = src[min((int)threadIdx.x + it * NT, N - 1)];
    }
    __device__ __forceinline__ void store(T *dst) const
    {
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int i = (int)threadIdx.x + it * NT;
            if (i < N) dst[i] = r[it];
        }
    }
};

// Positivity limiter (section 4) of one cell from the running bounds of its
// stored face-point increments; both half-waves of the cell call it and get
// the same factors.
template <int D, int R, typename PT>
__device__ __forceinline__ void limiter_factors(const double (*tile)[MCfg<D, R>::HN], const PT *ptile, int lc, int hf,
                                                const double *ref, bool active, bool ok, const IncBounds &bnd,
                                                const Limiter &lim, const Geom &g, const float *__restrict__ inc,
                                                long cell, int *__restrict__ err, double &th_rho, double &th_p)
{
    using C = MCfg<D, R>;
    constexpr int NV = D + 2, NPTS = C::S::NPTS;
    const double gam = g.gamma;
    th_rho = 1.0;
    th_p = 1.0;
    // bounds over the 3^d block; the two half-waves take alternate neighbours
    double rmax = -INFINITY, rmin = INFINITY, pmin = INFINITY, c2min = INFINITY;
    const bool flat = lim.flat_k1 > 0.0;
    constexpr int NB = D == 3 ? 27 : 9;
#pragma unroll
    for (int j = 0; j < (NB + 1) / 2; ++j) {
        const int nA = 2 * j, nB = 2 * j + 1 < NB ? 2 * j + 1 : 2 * j;
        const int oA = nA % 3 - 1 + C::HX * ((nA / 3) % 3 - 1 + C::HY * (D == 3 ? nA / 9 - 1 : 0));
        const int oB = nB % 3 - 1 + C::HX * ((nB / 3) % 3 - 1 + C::HY * (D == 3 ? nB / 9 - 1 : 0));
        const int o = lc + (hf ? oB : oA);
        const double r = tile[0][o];
        rmax = fmax(rmax, r);
        rmin = fmin(rmin, r);
        pmin = fmin(pmin, (double)ptile[o]);
        if (flat) c2min = fmin(c2min, gam * (double)ptile[o] / r);
    }
    rmax = pair_max(rmax);
    rmin = pair_min(rmin);
    pmin = pair_min(pmin);
    if (!(pmin > 0.0) && active) *err = ERR_NONPHYSICAL;   // a neighbour is not admissible
    // bounds widened by kappa (1 - eta)
    double f = lim.kappa;
    if (flat) {
        c2min = pair_min(c2min);
        f = lim.kappa * (1.0 - flattener_eta(undivided_divergence<D>(tile, lc, C::HX, C::HX * C::HY), c2min,
                                             lim.flat_k1));
    }
    rmax *= 1.0 + f;
    rmin *= 1.0 - f;
    pmin *= 1.0 - f;
    bool exact = false;
    if (active && ok) {
        // density scaling (eq. ppThetaRho) from the extreme point values: the
        // smallest ratio of each violated side is taken at its extreme point
        const double r0 = ref[0];
        const double rs_lo = r0 + (double)bnd.rlo, rs_hi = r0 + (double)bnd.rhi;
        if (rs_lo < rmin) th_rho = fmin(th_rho, (r0 - rmin) / (r0 - rs_lo));
        if (rs_hi > rmax) th_rho = fmin(th_rho, (rmax - r0) / (rs_hi - r0));
        // pressure at a point, exactly: p = p~ + th dw_p - (gamma-1)/2 th^2 rho~^2 |dw_u|^2 / rho
        // (dw: its increments in reconstruction variables).  With the least
        // dw_p and rho and the largest |dw_u|^2 this bounds every point from
        // below; only a cell whose bound falls under pmin takes the per-point
        // test and bisection (eq. thetapRoot, eq. thetaP).
        const double rlo = r0 + th_rho * (double)bnd.rlo;
        const double plow = pressure<D>(ref, gam) + th_rho * (double)bnd.plo -
                            0.5 * (gam - 1.0) * th_rho * th_rho * r0 * r0 * (double)bnd.v2 * rcp64(rlo);
        exact = !(rlo > 0.0 && plow >= pmin);
    }
    if (exact) {
        PhiInv<D> pi;
        pi.init(ref, gam);
        // this lane's face points: tau with bit 2 equal to hf (the ones it stored)
#pragma unroll 1
        for (int tau = 4 * hf; tau < NPTS; tau = (tau & 3) == 3 ? tau + 5 : tau + 1) {
            double w[NV], d[NV], u[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) w[v] = (double)inc[inc_index(tau, v, NV, g.ncell) + 4 * cell];
            pi.apply(w, d);
#pragma unroll
            for (int v = 0; v < NV; ++v) u[v] = ref[v] + th_rho * d[v];
            if (pressure<D>(u, gam) >= pmin) continue;
            double lo = 0.0, hi = 1.0;
#pragma unroll 1
            for (int it = 0; it < 60; ++it) {
                const double m = 0.5 * (lo + hi);
                double um[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) um[v] = ref[v] + m * th_rho * d[v];
                if (pressure<D>(um, gam) >= pmin) lo = m; else hi = m;
            }
            th_p = fmin(th_p, lo);
        }
    }
    th_p = pair_min(th_p);
}

template <int D, int R, bool BF, bool GATE>
__global__ __launch_bounds__((MixCfg<D, R>::NT)) void k_recon_mixed(
    const double *__restrict__ U, const uint4 *__restrict__ Afull, const uint4 *__restrict__ Alin,
    float *__restrict__ inc, double *__restrict__ theta, int *__restrict__ err, const uint8_t *__restrict__ flags,
    Geom g, Limiter lim, int sw, GateArgs ga)
{
    using C = MCfg<D, R>;
    using M = MixCfg<D, R>;
    constexpr int NV = C::NV;
    __shared__ double tile[NV][C::HN];
    __shared__ double ptile[C::HN];      // pressure of each tile cell, -1 where not admissible
    __shared__ uint4 As[M::A_FULL];
    __shared__ uint4 Al[M::A_LIN];
    __shared__ uint4 Wg[GATE ? GateShape<D>::SLOTS : 1];
    __shared__ __align__(16) float gvec[GATE ? GVEC_SIZE : 4];

    const int nbx = (g.n[0] + C::TX - 1) / C::TX, nby = (g.n[1] + C::TY - 1) / C::TY;
    const int nbz = D == 3 ? (g.n[2] + C::TZ - 1) / C::TZ : 1;
    const long nblk = (long)nbx * nby * nbz;
    const long tb = xcd_tile(blockIdx.x, nblk);
    if (tb >= nblk) return;
    const int bx = (int)(tb % nbx), by = (int)((tb / nbx) % nby), bz = (int)(tb / ((long)nbx * nby));
    const double gam = g.gamma;

    // prologue: the tile's loads into registers and the operand tables' loads
    // straight into LDS all in flight, then the tile's LDS stores (the GELU
    // chords are computed meanwhile)
    const int x0 = bx * C::TX - R, y0 = by * C::TY - R, z0 = D == 3 ? bz * C::TZ - R : 0;
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    TileLoad<D, R, M::NT> tl;
    tl.issue(U, g, x0, y0, z0);
    lds_rows<M::A_FULL, M::NT / 64>(Afull, As, wv, ln);
    lds_rows<M::A_LIN, M::NT / 64>(Alin, Al, wv, ln);
    LdsCopy<GATE ? 97 : 1, M::NT, float> cV;
    if constexpr (GATE) {
        lds_rows<GateShape<D>::SLOTS, M::NT / 64>(ga.w, Wg, wv, ln);
        cV.load(ga.vec);
        gelu_table_fill(gvec, threadIdx.x, M::NT);
    }
    tl.commit(U, g, lim, x0, y0, z0, tile, ptile);
    if constexpr (GATE) cV.store(gvec);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, hf = lane >> 5;
    const int ci = wave * 32 + (lane & 31);
    const int tx = ci % C::TX, ty = (ci / C::TX) % C::TY, tz = ci / (C::TX * C::TY);
    const int cx = bx * C::TX + tx, cy = by * C::TY + ty, cz = D == 3 ? bz * C::TZ + tz : 0;
    const bool active = cx < g.n[0] && cy < g.n[1] && (D == 2 || cz < g.n[2]);
    const long cell = active ? cx + (long)g.n[0] * (cy + (long)g.n[1] * cz) : 0;
    const uint32_t co = (uint32_t)cell;
    const int lc = (tx + R) + C::HX * ((ty + R) + C::HY * (D == 3 ? tz + R : 0));

    // precomputed decisions (two-pass indicator, replay), bit K for variable
    // K, all loaded before the first face-increment store: a wait for a load
    // issued after the stores would also wait for them (loads and stores share
    // the vector-memory counter); -1: WENO-AO everywhere
    int wbits = -1;
    if (flags) {
        int m = 0;
#pragma unroll
        for (int v = 0; v < NV; ++v) m |= (at4(flags, (long)v * g.ncell, co) != 0 ? 1 : 0) << v;
        wbits = m;
    }

    double ref[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) ref[v] = tile[v][lc];
    const bool ok = admissible<D>(ref, gam);
    if (!ok && active) *err = ERR_NONPHYSICAL;
    PhiRows<D> ph;
    ph.init(ref, gam);
    // every lane of the wave takes part in the matrix-core work; inactive and
    // non-physical cells compute on their (finite or not) data and store nothing
    IncBounds bnd;
    // flatness thresholds: 2^-40 of the natural scales of the reconstruction
    // variables (density, sound speed, pressure)
    float wsc[3] = {(float)(FLAT_REL * ref[0]), 0.f, 0.f};
    if constexpr (GATE) {
        const double pc = pressure<D>(ref, gam);
        wsc[1] = (float)(FLAT_REL * sqrt(fabs(gam * pc * ph.inv_rho)));
        wsc[2] = (float)(FLAT_REL * pc);
    }
    mixed_all_vars<D, R, BF, GATE>(tile, lc, lane, As, Al, ph, wbits, inc, co, g.ncell, active && ok, sw, Wg, gvec,
                                   ga.thr, ga.flags_out, wsc, bnd, std::make_integer_sequence<int, NV>{});

    double th_rho = 1.0, th_p = 1.0;
    settle_bounds(bnd);
    if (lim.on) {
        // the cell's averages read again from LDS through an opaque index, so
        // that nothing derived from them (its pressure) is held in registers,
        // or spilled, across the variables
        int l2 = lc;
        asm volatile("" : "+v"(l2));
        double r2[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) r2[v] = tile[v][l2];
        limiter_factors<D, R>(tile, ptile, lc, hf, r2, active, ok, bnd, lim, g, inc, cell, err, th_rho, th_p);
    }
    if (active && hf == 0) {
        theta[cell] = th_rho;
        theta[g.ncell + cell] = th_p;
    }
}

// --------------------------------------------------- streamed tables (3D R3) ---
// The interleaved operand table of the 3D R = 3 reconstruction (19 tiles of 8
// k-steps, ~311 KB) does not fit LDS.  It stays in global memory (L2-resident:
// every block reads the same bytes) and passes through a double-buffered LDS
// window of two tiles, loaded straight into LDS (global_load_lds_dwordx4)
// while the previous pair is in use.  Per variable the block first agrees
// whether any of its waves needs WENO-AO; if none does, only the S0 face-point
// table (two tiles) passes through.
// The learned gate on its own, for the streamed reconstruction: per cell the
// network on the radius-2 sphere of every variable (the inputs and rules of the
// fused gate), the decisions as bits of one byte per cell.
template <int D, int K>
__device__ __forceinline__ int gate_bit(const double (*tile)[MCfg<D, 2>::HN], int lc, int lane, const PhiRows<D> &ph,
                                        const uint4 *Wg, const float *gvec, float thr, const float (&wsc)[3])
{
    using C = MCfg<D, 2>;
    constexpr int KS = MixCfg<D, 2>::KS;
    static_assert(KS == GateShape<D>::KSG, "the gate reads the radius-2 contraction slots");
    const int hf = lane >> 5;
    const double Wc = w_component<D, K, C::HN>(tile, lc, ph);
    double dl[KS][8];
    double amax = 0.0;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            dl[ks][i] = slot_increment<D, 2, K>(tile, lc, hf, 16 * ks + i, 16 * ks + 8 + i, ph, Wc);
            amax = fmax(amax, fabs(dl[ks][i]));
        }
    amax = pair_max(amax);
    int ex = 0;
    if (amax > 0.0) frexp(amax, &ex);
    const double sc = ldexp(1.0, SB + 1 - max(ex, E_MIN_D + 1));
    uint4 xb[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        float y[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) y[i] = (float)(dl[ks][i] * sc);
        xb[ks] = make_uint4(pack_bf16(y[0], y[1]), pack_bf16(y[2], y[3]), pack_bf16(y[4], y[5]), pack_bf16(y[6], y[7]));
    }
    const float logit = gate_forward<D>(xb, lane, Wg, gvec);
    return logit > thr && amax > (double)wsc[K == 0 ? 0 : (K <= D ? 1 : 2)] ? 1 << K : 0;
}

template <int D, int... K>
__device__ __forceinline__ int gate_bits(const double (*tile)[MCfg<D, 2>::HN], int lc, int lane, const PhiRows<D> &ph,
                                         const uint4 *Wg, const float *gvec, float thr, const float (&wsc)[3],
                                         std::integer_sequence<int, K...>)
{
    return (gate_bit<D, K>(tile, [&] { int l = lc; asm volatile("" : "+v"(l)); return l; }(), lane, ph, Wg, gvec, thr,
                           wsc) | ...);
}

template <int D>
__global__ __launch_bounds__((MixCfg<D, 2>::NT)) void k_gate_flags(const double *__restrict__ U, Geom g, GateArgs ga)
{
    using C = MCfg<D, 2>;
    using M = MixCfg<D, 2>;
    constexpr int NV = C::NV;
    __shared__ double tile[NV][C::HN];
    __shared__ uint4 Wg[GateShape<D>::SLOTS];
    __shared__ __align__(16) float gvec[GVEC_SIZE];

    const int nbx = (g.n[0] + C::TX - 1) / C::TX, nby = (g.n[1] + C::TY - 1) / C::TY;
    const int nbz = D == 3 ? (g.n[2] + C::TZ - 1) / C::TZ : 1;
    const long nblk = (long)nbx * nby * nbz;
    const long tb = xcd_tile(blockIdx.x, nblk);
    if (tb >= nblk) return;
    const int bx = (int)(tb % nbx), by = (int)((tb / nbx) % nby), bz = (int)(tb / ((long)nbx * nby));
    const double gam = g.gamma;
    const Limiter off{0, 0.0, 0.0};
    load_tile<D, 2, M::NT>(U, g, off, bx * C::TX - 2, by * C::TY - 2, D == 3 ? bz * C::TZ - 2 : 0, tile,
                           (double *)nullptr);
    for (int i = threadIdx.x; i < GateShape<D>::SLOTS; i += M::NT) Wg[i] = ga.w[i];
    for (int i = threadIdx.x; i < 97; i += M::NT) gvec[i] = ga.vec[i];
    gelu_table_fill(gvec, threadIdx.x, M::NT);
    __syncthreads();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, hf = lane >> 5;
    const int ci = wave * 32 + (lane & 31);
    const int tx = ci % C::TX, ty = (ci / C::TX) % C::TY, tz = ci / (C::TX * C::TY);
    const int cx = bx * C::TX + tx, cy = by * C::TY + ty, cz = D == 3 ? bz * C::TZ + tz : 0;
    const bool active = cx < g.n[0] && cy < g.n[1] && (D == 2 || cz < g.n[2]);
    const long cell = active ? cx + (long)g.n[0] * (cy + (long)g.n[1] * cz) : 0;
    const int lc = (tx + 2) + C::HX * ((ty + 2) + C::HY * (D == 3 ? tz + 2 : 0));
    double ref[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) ref[v] = tile[v][lc];
    PhiRows<D> ph;
    ph.init(ref, gam);
    const double pc = pressure<D>(ref, gam);
    const float wsc[3] = {(float)(FLAT_REL * ref[0]), (float)(FLAT_REL * sqrt(fabs(gam * pc * ph.inv_rho))),
                          (float)(FLAT_REL * pc)};
    int bits = gate_bits<D>(tile, lc, lane, ph, Wg, gvec, ga.thr, wsc, std::make_integer_sequence<int, NV>{});
    if (!admissible<D>(ref, gam)) bits = (1 << NV) - 1;    // non-physical: WENO-AO (and reported by the reconstruction)
    if (active && hf == 0) ga.raw[cell] = (uint8_t)bits;
}

template <int D, int R>
struct StreamCfg {
    using M = MixCfg<D, R>;
    static constexpr int PH = 2;                              // tiles per phase
    static constexpr int TSL = M::KS * 2 * 64;                // 16-byte slots per tile (hi and lo)
    static constexpr int NPD = (M::NTF - M::TD_BEGIN + PH - 1) / PH;   // derivative-row phases
    static constexpr int NPP = (M::TP_END + PH - 1) / PH;     // point-row phases
};

// queue tiles [t0, min(t0 + PH, tend)) of table A into LDS buffer dst; every
// wave copies whole 64-slot rows, one 16-byte slot per lane
template <int D, int R>
__device__ __forceinline__ void stream_tiles(const uint4 *__restrict__ A, int t0, int tend, uint4 *dst)
{
    using SC = StreamCfg<D, R>;
    constexpr int NW = MixCfg<D, R>::NT / 64;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n = (tend - t0 < SC::PH ? tend - t0 : SC::PH);
    const int rows = n * SC::TSL / 64;
    typedef __attribute__((address_space(1))) void *gptr;
    typedef __attribute__((address_space(3))) void *lptr;
    for (int r = wave; r < rows; r += NW)
        __builtin_amdgcn_global_load_lds((gptr)(A + (long)t0 * SC::TSL + r * 64 + lane), (lptr)(dst + r * 64), 16, 0,
                                         0);
}

// this wave's own direct-to-LDS loads (and every other memory operation) done,
// then every wave's
__device__ __forceinline__ void stream_wait()
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

template <int D, int R, int K, bool BF>
__device__ __forceinline__ void mixed_var_stream(const double (*tile)[MCfg<D, R>::HN], int lc, int lane,
                                                 const uint4 *__restrict__ Afull, const uint4 *__restrict__ Alin,
                                                 uint4 (*buf)[StreamCfg<D, R>::PH * StreamCfg<D, R>::TSL],
                                                 const PhiRows<D> &ph, int fbits,
                                                 int gbits, uint8_t *__restrict__ fl_out, float *__restrict__ inc,
                                                 uint32_t co, long ncell, bool active, int sw, IncBounds &bnd)
{
    using C = MCfg<D, R>;
    using M = MixCfg<D, R>;
    using SC = StreamCfg<D, R>;
    using S = typename C::S;
    constexpr int NV = C::NV, NST = S::NST, NPTS = S::NPTS, NROWS = S::NROWS, KS = M::KS;
    const int hf = lane >> 5;
    const double Wc = w_component<D, K, C::HN>(tile, lc, ph);

    // increments over this lane's slots 16 ks + 8 hf + i, rounded to float32
    // once (scaling by a power of two afterwards is exact)
    float ys[KS][8];
    float amax = 0.f;
    int lcc = lc;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            ys[ks][i] = (float)slot_increment<D, R, K>(tile, lcc, hf, 16 * ks + i, 16 * ks + 8 + i, ph, Wc);
            asm volatile("" : "+v"(ys[ks][i]));
            amax = fmaxf(amax, fabsf(ys[ks][i]));
        }
        asm volatile("" : "+v"(lcc) : "v"(ys[ks][7]));
    }
    amax = pair_max(amax);
    int ex = 0;
    if (amax > 0.f) frexpf(amax, &ex);         // amax in [2^(ex-1), 2^ex)
    const int e = max(ex - 1, E_MIN_F);
    const int ue = e - SB - sw;                  // accumulator units: value = acc * 2^ue
    uint4 bh[KS], bl[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        uint32_t h[4], l[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            split_pair<BF>(ldexpf(ys[ks][2 * i], SB - e), ldexpf(ys[ks][2 * i + 1], SB - e), h[i], l[i]);
        bh[ks] = make_uint4(h[0], h[1], h[2], h[3]);
        bl[ks] = make_uint4(l[0], l[1], l[2], l[3]);
    }

    // gate decisions (dilated over the 3^3 block, gbits >= 0; recorded in
    // fl_out), else the precomputed decisions (fbits >= 0), else WENO-AO
    const bool use_weno = gbits >= 0 ? ((gbits >> K) & 1) != 0 : (fbits >= 0 ? ((fbits >> K) & 1) != 0 : true);
    if (gbits >= 0 && active && hf == 0) at4(fl_out, (long)K * ncell, co) = use_weno ? 1 : 0;
    const uint32_t lo16 = co * 16u + (uint32_t)hf * (uint32_t)(16 * ncell);
    float v2k = 0.f;
    const bool wave_weno = __any(use_weno && active);
    if (__syncthreads_or(wave_weno)) {
        float bp[4] = {0.f, 0.f, 0.f, 0.f};
        float cm[4] = {hf == 0 ? 1.f : 0.f, 0.f, 0.f, 0.f};
        constexpr int NPH = SC::NPD + SC::NPP;
        stream_tiles<D, R>(Afull, M::TD_BEGIN, M::NTF, buf[0]);
#pragma unroll 1
        for (int p = 0; p < NPH; ++p) {
            stream_wait();
            if (p + 1 < NPH) {
                const int q = p + 1;
                if (q < SC::NPD) stream_tiles<D, R>(Afull, M::TD_BEGIN + SC::PH * q, M::NTF, buf[q & 1]);
                else stream_tiles<D, R>(Afull, SC::PH * (q - SC::NPD), M::TP_END, buf[q & 1]);
            }
            const uint4 *As = buf[p & 1];
            if (p < SC::NPD) {
                // smoothness indicators: derivative tiles of this phase
                if (wave_weno) {
#pragma unroll
                    for (int tt = 0; tt < SC::PH; ++tt) {
                        const int t = M::TD_BEGIN + SC::PH * p + tt;
                        if (t < M::NTF) {
                            f16v acc = {};
#pragma unroll
                            for (int ks = 0; ks < KS; ++ks) {
                                const uint4 ah = As[((tt * KS + ks) * 2 + 0) * 64 + lane];
                                const uint4 al = As[((tt * KS + ks) * 2 + 1) * 64 + lane];
                                acc = mfma<BF>(ah, bh[ks], acc);
                                acc = mfma<BF>(ah, bl[ks], acc);
                                acc = mfma<BF>(al, bh[ks], acc);
                            }
#pragma unroll
                            for (int j = 0; j < 16; ++j) {
                                const int tau = 4 * t + j / 4;
                                if (tau >= NPTS && tau < NROWS) bp[j % 4] += acc[j] * acc[j];
                            }
                        }
                    }
                }
                if (p == SC::NPD - 1 && wave_weno) {
                    // nonlinear weights (eq. nlinWts) in FP64 and WENO-AO
                    // coefficients (eq. wenoAOrec); linear cells keep stencil 0
                    double om[4], part = 0.0;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int q = 4 * hf + i;
                        const double beta = ldexp((double)bp[i], 2 * ue);
                        om[i] = q < NST ? lin_w<D>(q) * rcp64(beta * beta + EPS_WENO) : 0.0;
                        part += om[i];
                    }
                    const double inv = rcp64(pair_sum(part));
#pragma unroll
                    for (int i = 0; i < 4; ++i) om[i] *= inv;
                    const double om0 = lower_half(om[0]);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int q = 4 * hf + i;
                        double cq = q == 0 ? om0 * inv_lin0<D>() : (q < NST ? om[i] - om0 * lin_ratio<D>(q) : 0.0);
                        if (!use_weno) cq = q == 0 ? 1.0 : 0.0;
                        cm[i] = (float)cq;
                    }
                }
            } else {
                // blended face-point increments of this phase's point tiles, in
                // pairs (a phase holds an even number of tiles)
                static_assert(SC::PH % 2 == 0, "point tiles are blended in pairs");
#pragma unroll
                for (int tt = 0; tt < SC::PH; tt += 2) {
                    const int t = SC::PH * (p - SC::NPD) + tt;
                    if (t < M::TP_END) {
                        f16v acc0 = {}, acc1 = {};
#pragma unroll
                        for (int ks = 0; ks < KS; ++ks) {
                            const uint4 ah = As[((tt * KS + ks) * 2 + 0) * 64 + lane];
                            const uint4 al = As[((tt * KS + ks) * 2 + 1) * 64 + lane];
                            acc0 = mfma<BF>(ah, bh[ks], acc0);
                            acc0 = mfma<BF>(ah, bl[ks], acc0);
                            acc0 = mfma<BF>(al, bh[ks], acc0);
                        }
                        if (t + 1 < M::TP_END) {
#pragma unroll
                            for (int ks = 0; ks < KS; ++ks) {
                                const uint4 ah = As[(((tt + 1) * KS + ks) * 2 + 0) * 64 + lane];
                                const uint4 al = As[(((tt + 1) * KS + ks) * 2 + 1) * 64 + lane];
                                acc1 = mfma<BF>(ah, bh[ks], acc1);
                                acc1 = mfma<BF>(ah, bl[ks], acc1);
                                acc1 = mfma<BF>(al, bh[ks], acc1);
                            }
                        }
                        float grp[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int gq = 0; gq < 4; ++gq) {
                            if (4 * t + gq < NPTS) {
                                float p0 = 0.f, p1 = 0.f;
#pragma unroll
                                for (int i = 0; i < 4; ++i) {
                                    p0 += cm[i] * acc0[4 * gq + i];
                                    p1 += cm[i] * acc1[4 * gq + i];
                                }
                                grp[gq] = ldexpf(pair_blend(p0, p1, hf), ue);
                                if (4 * (t + hf) + gq < NPTS) note_increment<D, K>(bnd, grp[gq], v2k);
                            }
                        }
                        if (active)
                            store_group<NV, K>(inc, 4 * t, ncell, lo16, make_float4(grp[0], grp[1], grp[2], grp[3]));
                    }
                }
            }
        }
    } else {
        // no wave of the block needs WENO-AO for this variable: S0 face rows only
        stream_tiles<D, R>(Alin, 0, M::NTL, buf[0]);
        stream_wait();
        const uint4 *Al = buf[0];
#pragma unroll
        for (int t = 0; t < M::NTL; ++t) {
            f16v acc = {};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const uint4 ah = Al[((t * KS + ks) * 2 + 0) * 64 + lane];
                const uint4 al = Al[((t * KS + ks) * 2 + 1) * 64 + lane];
                acc = mfma<BF>(ah, bh[ks], acc);
                acc = mfma<BF>(ah, bl[ks], acc);
                acc = mfma<BF>(al, bh[ks], acc);
            }
#pragma unroll
            for (int G = 0; G < 4; ++G) {
                // registers 4 G .. 4 G + 3 hold points T0 .. T0 + 3 in the lower
                // half-wave, T0 + 4 .. T0 + 7 in the upper
                const int T0 = 32 * t + 8 * G;
                if (T0 < NPTS) {
                    float grp[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        grp[i] = ldexpf(acc[4 * G + i], ue);
                        if (T0 + i + 4 < NPTS || (hf == 0 && T0 + i < NPTS)) note_increment<D, K>(bnd, grp[i], v2k);
                    }
                    if (active) store_group<NV, K>(inc, T0, ncell, lo16, make_float4(grp[0], grp[1], grp[2], grp[3]));
                }
            }
        }
    }
    // the buffers are free again only when every wave is done with them
    __syncthreads();
    if constexpr (K >= 1 && K <= D) bnd.v2 += pair_max(v2k);
}

template <int D, int R, bool BF, int... K>
__device__ __forceinline__ void mixed_all_vars_stream(const double (*tile)[MCfg<D, R>::HN], int lc, int lane,
                                                      const uint4 *Afull, const uint4 *Alin,
                                                      uint4 (*buf)[StreamCfg<D, R>::PH * StreamCfg<D, R>::TSL],
                                                      const PhiRows<D> &ph, int fbits, int gbits,
                                                      uint8_t *fl_out, float *inc, uint32_t co, long ncell,
                                                      bool active, int sw, IncBounds &bnd,
                                                      std::integer_sequence<int, K...>)
{
    ((mixed_var_stream<D, R, K, BF>(tile, [&] { int l = lc; asm volatile("" : "+v"(l)); return l; }(), lane, Afull,
                                    Alin, buf, ph, fbits, gbits, fl_out, inc, co, ncell, active, sw, bnd)),
     ...);
}

template <int D, int R, bool BF, bool GATE>
__global__ __launch_bounds__((MixCfg<D, R>::NT)) void k_recon_mixed_stream(
    const double *__restrict__ U, const uint4 *__restrict__ Afull, const uint4 *__restrict__ Alin,
    float *__restrict__ inc, double *__restrict__ theta, int *__restrict__ err, const uint8_t *__restrict__ flags,
    Geom g, Limiter lim, int sw, GateArgs ga)
{
    using C = MCfg<D, R>;
    using M = MixCfg<D, R>;
    using SC = StreamCfg<D, R>;
    constexpr int NV = C::NV;
    // the gate's per-cell decision bits over the tile and a one-cell halo
    constexpr int GX = C::TX + 2, GY = C::TY + 2, GZ = D == 3 ? C::TZ + 2 : 1;
    __shared__ double tile[NV][C::HN];
    __shared__ float ptile[C::HN];       // pressure of each tile cell, -1 where not admissible
    __shared__ uint4 buf[2][SC::PH * SC::TSL];
    __shared__ uint8_t gtile[GATE ? GX * GY * GZ : 1];

    const int nbx = (g.n[0] + C::TX - 1) / C::TX, nby = (g.n[1] + C::TY - 1) / C::TY;
    const int nbz = D == 3 ? (g.n[2] + C::TZ - 1) / C::TZ : 1;
    const long nblk = (long)nbx * nby * nbz;
    const long tb = xcd_tile(blockIdx.x, nblk);
    if (tb >= nblk) return;
    const int bx = (int)(tb % nbx), by = (int)((tb / nbx) % nby), bz = (int)(tb / ((long)nbx * nby));
    const double gam = g.gamma;

    load_tile<D, R, M::NT>(U, g, lim, bx * C::TX - R, by * C::TY - R, D == 3 ? bz * C::TZ - R : 0, tile, ptile);
    if constexpr (GATE) {
        for (int i = threadIdx.x; i < GX * GY * GZ; i += M::NT) {
            const int hx = i % GX, hy = (i / GX) % GY, hz = i / (GX * GY);
            // (past a non-periodic boundary: the decisions of the cell the ghost copies)
            const int gx = ghost_index(g, 0, bx * C::TX - 1 + hx), gy = ghost_index(g, 1, by * C::TY - 1 + hy);
            const int gz = D == 3 ? ghost_index(g, 2, bz * C::TZ - 1 + hz) : 0;
            gtile[i] = ga.raw[gx + (long)g.n[0] * (gy + (long)g.n[1] * gz)];
        }
    }
    __syncthreads();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, hf = lane >> 5;
    const int ci = wave * 32 + (lane & 31);
    const int tx = ci % C::TX, ty = (ci / C::TX) % C::TY, tz = ci / (C::TX * C::TY);
    const int cx = bx * C::TX + tx, cy = by * C::TY + ty, cz = D == 3 ? bz * C::TZ + tz : 0;
    const bool active = cx < g.n[0] && cy < g.n[1] && (D == 2 || cz < g.n[2]);
    const long cell = active ? cx + (long)g.n[0] * (cy + (long)g.n[1] * cz) : 0;
    const uint32_t co = (uint32_t)cell;
    const int lc = (tx + R) + C::HX * ((ty + R) + C::HY * (D == 3 ? tz + R : 0));

    // a variable takes WENO-AO when the network marks it troubled in any cell
    // of the 3^d block: the radius-2 inputs of the neighbours together see the
    // radius-3 stencil
    int gbits = -1;
    if constexpr (GATE) {
        const int lg = (tx + 1) + GX * ((ty + 1) + GY * (D == 3 ? tz + 1 : 0));
        int m = 0;
#pragma unroll
        for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) m |= gtile[lg + dx + GX * (dy + GY * dz)];
        gbits = m;
    }
    // precomputed decisions (two-pass indicator, replay), bit K for variable
    // K, loaded before the first face-increment store (see k_recon_mixed);
    // -1: none
    int fbits = -1;
    if (flags) {
        int m = 0;
#pragma unroll
        for (int v = 0; v < NV; ++v) m |= (at4(flags, (long)v * g.ncell, co) != 0 ? 1 : 0) << v;
        fbits = m;
    }

    double ref[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) ref[v] = tile[v][lc];
    const bool ok = admissible<D>(ref, gam);
    if (!ok && active) *err = ERR_NONPHYSICAL;
    PhiRows<D> ph;
    ph.init(ref, gam);
    IncBounds bnd;
    mixed_all_vars_stream<D, R, BF>(tile, lc, lane, Afull, Alin, buf, ph, fbits, gbits, ga.flags_out, inc, co,
                                    g.ncell, active && ok, sw, bnd, std::make_integer_sequence<int, NV>{});

    double th_rho = 1.0, th_p = 1.0;
    settle_bounds(bnd);
    if (lim.on)
        limiter_factors<D, R>(tile, ptile, lc, hf, ref, active, ok, bnd, lim, g, inc, cell, err, th_rho, th_p);
    if (active && hf == 0) {
        theta[cell] = th_rho;
        theta[g.ncell + cell] = th_p;
    }
}

// ------------------------------------------------------------------- flux ---
template <int D, int R, int A>
__device__ __forceinline__ void lower_face_flux_mixed(const double *__restrict__ U, const float *__restrict__ inc,
                                                      const double *__restrict__ theta, const Geom &g, long cell,
                                                      long lower, const double *refR, const PhiInv<D> &piR,
                                                      double thR, int hll, double *Fbar)
{
    using S = Stencil<D, R>;
    constexpr int NV = D + 2, NG = S::NG;
    double refL[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) refL[v] = U[v * g.ncell + lower];
    const double thL = theta[lower] * theta[g.ncell + lower];
    PhiInv<D> piL;
    piL.init(refL, g.gamma);
    const float *incL = inc + 4 * lower, *incR = inc + 4 * cell;
#pragma unroll
    for (int v = 0; v < NV; ++v) Fbar[v] = 0.0;
    // four Gauss points per face (3D R = 2): each side's face is one vector per
    // variable, loaded at once (the loop is unrolled: the vectors' lanes are
    // compile-time indices)
    constexpr bool VEC = NG == 4;
    float4 gL[VEC ? NV : 1], gR[VEC ? NV : 1];
    if constexpr (VEC) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            gL[v] = *reinterpret_cast<const float4 *>(incL + inc_index((2 * A + 1) * NG, v, NV, g.ncell));
            gR[v] = *reinterpret_cast<const float4 *>(incR + inc_index((2 * A + 0) * NG, v, NV, g.ncell));
        }
    }
    // other point counts (2D; 3D R = 3: nine): each side's points lie in 16-byte
    // groups of four (inc_index); a group is loaded, one vector per variable,
    // at the first point that falls in it, so one group per side is live
    constexpr bool GRP = NG != 4;
    float4 cL[GRP ? NV : 1], cR[GRP ? NV : 1];
    constexpr int UNROLL = VEC || GRP ? NG : 1;
#pragma unroll UNROLL
    for (int gi = 0; gi < NG; ++gi) {
        double wL[NV], wR[NV], dL[NV], dR[NV], uL[NV], uR[NV], F[NV];
        if constexpr (GRP) {
            const int tL = (2 * A + 1) * NG + gi, tR = (2 * A + 0) * NG + gi;
            if (gi == 0 || (tL & 3) == 0) {
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    cL[v] = *reinterpret_cast<const float4 *>(incL + inc_index(tL & ~3, v, NV, g.ncell));
            }
            if (gi == 0 || (tR & 3) == 0) {
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    cR[v] = *reinterpret_cast<const float4 *>(incR + inc_index(tR & ~3, v, NV, g.ncell));
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                wL[v] = (double)cL[v][tL & 3];
                wR[v] = (double)cR[v][tR & 3];
            }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if constexpr (VEC) {
                wL[v] = (double)gL[v][gi];
                wR[v] = (double)gR[v][gi];
            } else if constexpr (!GRP) {
                wL[v] = (double)incL[inc_index((2 * A + 1) * NG + gi, v, NV, g.ncell)];
                wR[v] = (double)incR[inc_index((2 * A + 0) * NG + gi, v, NV, g.ncell)];
            }
        }
        piL.apply(wL, dL);
        piR.apply(wR, dR);
#pragma unroll
        for (int v = 0; v < NV; ++v) { uL[v] = refL[v] + thL * dL[v]; uR[v] = refR[v] + thR * dR[v]; }
        riemann<D, A, true>(uL, uR, g.gamma, hll, F);
        const double w = face_weight<D, R>(gi);
#pragma unroll
        for (int v = 0; v < NV; ++v) Fbar[v] += w * F[v];
    }
}

// Flux through the face of `cell` on this side of axis A when it lies on a
// non-periodic boundary: the cell's limited state inside, the state the
// boundary condition gives outside (section 5.3, step 4).
template <int D, int R, int A>
__device__ __forceinline__ void boundary_face_flux_mixed(const float *__restrict__ inc, const Geom &g, long cell,
                                                         int side, const double *ref, const PhiInv<D> &pi, double th,
                                                         int hll, double *Fbar)
{
    using S = Stencil<D, R>;
    constexpr int NV = D + 2, NG = S::NG;
    const float *incc = inc + 4 * cell;
#pragma unroll
    for (int v = 0; v < NV; ++v) Fbar[v] = 0.0;
#pragma unroll 1
    for (int gi = 0; gi < NG; ++gi) {
        double w[NV], d[NV], in[NV], out[NV], F[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) w[v] = (double)incc[inc_index((2 * A + side) * NG + gi, v, NV, g.ncell)];
        pi.apply(w, d);
#pragma unroll
        for (int v = 0; v < NV; ++v) in[v] = ref[v] + th * d[v];
        boundary_state<D>(g, A, side, in, out);
        if (side) riemann<D, A, true>(in, out, g.gamma, hll, F);
        else riemann<D, A, true>(out, in, g.gamma, hll, F);
        const double wt = face_weight<D, R>(gi);
#pragma unroll
        for (int v = 0; v < NV; ++v) Fbar[v] += wt * F[v];
    }
}

// The fluxes of axis A at `cell`: its lower face into fbar and, on an upper
// non-periodic boundary, its upper face into fbar_top.
template <int D, int R, int A>
__device__ __forceinline__ bool axis_fluxes_mixed(const double *__restrict__ U, const float *__restrict__ inc,
                                                  const double *__restrict__ theta, double *__restrict__ fbar,
                                                  double *__restrict__ fbar_top, long plane, const Geom &g, long cell,
                                                  const int *c, const double *refR, const PhiInv<D> &piR, double thR,
                                                  int hll)
{
    constexpr int NV = D + 2;
    double F[NV];
    bool ok = true;
    if (!g.periodic && c[A] == 0 && g.bc[A][0] != BC_PERIODIC) {
        boundary_face_flux_mixed<D, R, A>(inc, g, cell, 0, refR, piR, thR, hll, F);
    } else {
        int lc[3] = {c[0], c[1], c[2]};
        lc[A] = wrapi(c[A] - 1, g.n[A]);
        const long lower = lc[0] + (long)g.n[0] * (lc[1] + (long)g.n[1] * lc[2]);
        lower_face_flux_mixed<D, R, A>(U, inc, theta, g, cell, lower, refR, piR, thR, hll, F);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) { fbar[(A * NV + v) * g.ncell + cell] = F[v]; ok = ok && isfinite(F[v]); }
    if (!g.periodic && c[A] == g.n[A] - 1 && g.bc[A][1] != BC_PERIODIC) {
        boundary_face_flux_mixed<D, R, A>(inc, g, cell, 1, refR, piR, thR, hll, F);
        const long pi = plane_index(A, c[0], c[1], c[2], g.n);
#pragma unroll
        for (int v = 0; v < NV; ++v) { fbar_top[(A * NV + v) * plane + pi] = F[v]; ok = ok && isfinite(F[v]); }
    }
    return ok;
}

template <int D, int R>
__global__ __launch_bounds__(256) void k_flux_mixed(const double *__restrict__ U, const float *__restrict__ inc,
                                                    const double *__restrict__ theta, double *__restrict__ fbar,
                                                    double *__restrict__ fbar_top, long plane,
                                                    int *__restrict__ err, Geom g, int hll)
{
    constexpr int NV = D + 2;
    const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= g.ncell) return;
    const int cx = (int)(cell % g.n[0]), cy = (int)((cell / g.n[0]) % g.n[1]);
    const int cz = (int)(cell / ((long)g.n[0] * g.n[1]));
    double refR[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) refR[v] = U[v * g.ncell + cell];
    const double thR = theta[cell] * theta[g.ncell + cell];
    PhiInv<D> piR;
    piR.init(refR, g.gamma);
    const int c[3] = {cx, cy, cz};
    bool ok = axis_fluxes_mixed<D, R, 0>(U, inc, theta, fbar, fbar_top, plane, g, cell, c, refR, piR, thR, hll);
    ok = axis_fluxes_mixed<D, R, 1>(U, inc, theta, fbar, fbar_top, plane, g, cell, c, refR, piR, thR, hll) && ok;
    if constexpr (D == 3)
        ok = axis_fluxes_mixed<D, R, 2>(U, inc, theta, fbar, fbar_top, plane, g, cell, c, refR, piR, thR, hll) && ok;
    if (!ok) *err = ERR_NONPHYSICAL;
}

template <int D, int R>
__global__ __launch_bounds__(256) void k_states_mixed(const double *__restrict__ U, const float *__restrict__ inc,
                                                      const double *__restrict__ theta, double *__restrict__ states,
                                                      Geom g)
{
    using S = Stencil<D, R>;
    constexpr int NV = D + 2, NPTS = S::NPTS;
    const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= g.ncell) return;
    double ref[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) ref[v] = U[v * g.ncell + cell];
    const double th = theta[cell] * theta[g.ncell + cell];
    PhiInv<D> pi;
    pi.init(ref, g.gamma);
#pragma unroll 1
    for (int s = 0; s < NPTS; ++s) {
        double w[NV], d[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) w[v] = (double)inc[inc_index(s, v, NV, g.ncell) + 4 * cell];
        pi.apply(w, d);
#pragma unroll
        for (int v = 0; v < NV; ++v) states[(cell * NPTS + s) * NV + v] = ref[v] + th * d[v];
    }
}

template <int D, int R, bool BF>
hipError_t mixed_impl(const Geom &g, const MixTables &t, const Work &w, const Limiter &lim, int riemann,
                      const double *U0, const double *Uin, double *out, int stage, double dt, double *states,
                      hipStream_t s, const Timing &tm, const GateArgs &ga)
{
    using C = MCfg<D, R>;
    using M = MixCfg<D, R>;
    auto mark = [&](int kind, int begin) { if (tm.on) tm.record(tm.self, kind, s, begin); };
    const long nblk = (long)((g.n[0] + C::TX - 1) / C::TX) * ((g.n[1] + C::TY - 1) / C::TY) *
                      (D == 3 ? (g.n[2] + C::TZ - 1) / C::TZ : 1);
    const long grid = ((nblk + 7) / 8) * 8;
    mark(KT_RECON, 1);
    if constexpr (streamed_tables(D, R)) {
        if (ga.w) {
            using C2 = MCfg<D, 2>;
            const long nb2 = (long)((g.n[0] + C2::TX - 1) / C2::TX) * ((g.n[1] + C2::TY - 1) / C2::TY) *
                             ((g.n[2] + C2::TZ - 1) / C2::TZ);
            hipLaunchKernelGGL((k_gate_flags<D>), dim3((unsigned)(((nb2 + 7) / 8) * 8)), dim3(MixCfg<D, 2>::NT), 0, s,
                               Uin, g, ga);
            hipLaunchKernelGGL((k_recon_mixed_stream<D, R, BF, true>), dim3((unsigned)grid), dim3(M::NT), 0, s, Uin,
                               t.full, t.lin, w.inc32, w.theta, w.err, (const uint8_t *)nullptr, g, lim, t.sw, ga);
        } else {
            hipLaunchKernelGGL((k_recon_mixed_stream<D, R, BF, false>), dim3((unsigned)grid), dim3(M::NT), 0, s, Uin,
                               t.full, t.lin, w.inc32, w.theta, w.err, w.flags_in, g, lim, t.sw, ga);
        }
    } else {
        if (ga.w)
            hipLaunchKernelGGL((k_recon_mixed<D, R, BF, true>), dim3((unsigned)grid), dim3(M::NT), 0, s, Uin,
                               t.full, t.lin, w.inc32, w.theta, w.err, (const uint8_t *)nullptr, g, lim, t.sw, ga);
        else
            hipLaunchKernelGGL((k_recon_mixed<D, R, BF, false>), dim3((unsigned)grid), dim3(M::NT), 0, s, Uin,
                               t.full, t.lin, w.inc32, w.theta, w.err, w.flags_in, g, lim, t.sw, ga);
    }
    mark(KT_RECON, 0);
    const unsigned nb = (unsigned)((g.ncell + 255) / 256);
    if (states) {
        hipLaunchKernelGGL((k_states_mixed<D, R>), dim3(nb), dim3(256), 0, s, Uin, w.inc32, w.theta, states, g);
        return hipGetLastError();
    }
    mark(KT_FLUX, 1);
    hipLaunchKernelGGL((k_flux_mixed<D, R>), dim3(nb), dim3(256), 0, s, Uin, w.inc32, w.theta, w.fbar, w.fbar_top,
                       w.plane, w.err, g, riemann);
    mark(KT_FLUX, 0);
    mark(KT_UPDATE, 1);
    hipError_t e = launch_update(D, g, w, U0, Uin, out, stage, dt, s);
    mark(KT_UPDATE, 0);
    return e;
}

}  // namespace

bool mixed_supported(int dim, int R) { return (dim == 2 || dim == 3) && (R == 2 || R == 3); }

int gate_operand_slots(int dim) { return dim == 2 ? GateShape<2>::SLOTS : GateShape<3>::SLOTS; }

int gate_slot_input(int dim, int k)
{
    if (dim == 2) return k < 25 ? k : -1;
    return k < MixCfg<3, 2>::NK ? slot_point<3, 2>(k) : -1;
}

int gate_w1_exp(int dim) { return dim == 2 ? 0 : -(SB + 1); }

int mixed_operand_slots(int dim, int R, int which)
{
#define KF_SLOTS(d, r) return which == 0 ? MixCfg<d, r>::A_FULL : MixCfg<d, r>::A_LIN
    if (dim == 2 && R == 2) KF_SLOTS(2, 2);
    if (dim == 2 && R == 3) KF_SLOTS(2, 3);
    if (dim == 3 && R == 2) KF_SLOTS(3, 2);
    if (dim == 3 && R == 3) KF_SLOTS(3, 3);
#undef KF_SLOTS
    return -1;
}

hipError_t launch_rhs_mixed(int dim, int R, bool bf16, const Geom &g, const MixTables &t, const Work &w,
                            const Limiter &lim, int riemann, const double *U0, const double *Uin, double *out,
                            int stage, double dt, double *states, hipStream_t s, const Timing &tm, const GateArgs &ga)
{
#define KF_MIX(d, r)                                                                                              \
    return bf16 ? mixed_impl<d, r, true>(g, t, w, lim, riemann, U0, Uin, out, stage, dt, states, s, tm, ga)   \
                : mixed_impl<d, r, false>(g, t, w, lim, riemann, U0, Uin, out, stage, dt, states, s, tm, ga)
    if (dim == 2 && R == 2) KF_MIX(2, 2);
    if (dim == 2 && R == 3) KF_MIX(2, 3);
    if (dim == 3 && R == 2) KF_MIX(3, 2);
    if (dim == 3 && R == 3) KF_MIX(3, 3);
#undef KF_MIX
    return hipErrorInvalidValue;
}

}  // namespace kfvm
