// Adjoint of the rasterizer: gradients of a scalar loss with respect to the
// raw Gaussian parameters, given dL/dRGB.  The paper calls its rasterizer
// differentiable without giving the adjoint; this follows the usual
// replay of the blend from the saved per-pixel final transmittance and last
// contributor, with wavefront-reduced atomics (the DISTWAR approach the paper
// cites among related work).
//
// k_blend_bwd: one 256-thread workgroup per tile and one wavefront per 8 x 8
// quadrant, with the forward's staged coefficients and exponent (so both take
// the same contribution and clamp decisions).  Each pixel walks its tile list
// back to front from its last contributor:
//     T_n = T_{n+1} / (1 - a_n)
//     dL/dc_n     = g . a_n T_n                        (g = dL/dRGB of the pixel)
//     dL/da_n     = T_n g . (c_n - R_n),   R_{n-1} = c_n a_n + (1 - a_n) R_n,  R_last = bg
//     dL/dq_n     = -a_n / 2 dL/da_n     (0 where a_n is clamped at alpha_max)
// The per-pixel terms that depend on the Gaussian are summed over the
// wavefront with DPP, over the workgroup's four wavefronts with LDS atomics,
// and go to HBM with one atomic per Gaussian, batch and accumulator.
// Accumulators per Gaussian (planar, 9 planes):
//     0: sum dL/dq            1..3: sum dL/dq dx^2, dx dy, dy^2
//     4..5: sum dL/dq dx, dy  6..8: sum dL/dcolour
// From these, dL/dA, dL/dB, dL/dC, dL/du, dL/dv and dL/do (= -2 sum dL/dq / o,
// since da/do = a / o) follow per Gaussian.
//
// k_preprocess_bwd: one lane per Gaussian; recomputes the preprocessing
// steps in binary32 and applies the chain rule in reverse: conic = inverse
// of Sigma', Sigma' = T Sigma T^T + dilation I, T = J R_cam, Sigma = M M^T,
// M = R(q / |q|) diag(exp(log-scale)), (u, v) and J from the camera-space
// mean, opacity = sigmoid(logit), colour = max(0, SH . Y(d) + 1/2).
#include "fgs_internal.hpp"
#include "blend_common.hpp"
#include "sh_basis.hpp"

namespace fgs {
namespace {

constexpr int kWave = 64;
constexpr int kAcc = 9;

// ---- wavefront sum with DPP ----------------------------------------------
// Butterfly within each row of 16 lanes, then the row sums are carried by
// row_bcast:15 and row_bcast:31; lane 63 ends with the total.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_add(float v) {
    const int moved = __builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, kRowMask, 0xf, false);
    return v + __int_as_float(moved);
}

__device__ __forceinline__ void wave_sum_to_63(float *v) {
#pragma unroll
    for (int k = 0; k < kAcc; ++k) v[k] = dpp_add<0xb1, 0xf>(v[k]);   // quad_perm [1,0,3,2]
#pragma unroll
    for (int k = 0; k < kAcc; ++k) v[k] = dpp_add<0x4e, 0xf>(v[k]);   // quad_perm [2,3,0,1]
#pragma unroll
    for (int k = 0; k < kAcc; ++k) v[k] = dpp_add<0x124, 0xf>(v[k]);  // row_ror:4
#pragma unroll
    for (int k = 0; k < kAcc; ++k) v[k] = dpp_add<0x128, 0xf>(v[k]);  // row_ror:8
#pragma unroll
    for (int k = 0; k < kAcc; ++k) v[k] = dpp_add<0x142, 0xa>(v[k]);  // row_bcast:15 into rows 1, 3
#pragma unroll
    for (int k = 0; k < kAcc; ++k) v[k] = dpp_add<0x143, 0xc>(v[k]);  // row_bcast:31 into rows 2, 3
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)v, d, kWave);
        v = o > v ? o : v;
    }
    return v;
}

__global__ __launch_bounds__(kBlock) void k_blend_bwd(const GaussState *__restrict__ gs,
                                                      const uint32_t *__restrict__ values,
                                                      const uint2 *__restrict__ ranges, const float *__restrict__ Tfin,
                                                      const uint32_t *__restrict__ last, const float *__restrict__ dL,
                                                      int W, int H, int tiles_x, DevOptions op,
                                                      float *__restrict__ acc, int64_t acc_stride) {
    __shared__ float4 s_f0[kBlock], s_f1[kBlock];
    __shared__ float2 s_f2[kBlock];
    __shared__ uint32_t s_id[kBlock];
    __shared__ uint32_t s_rel[4][kBlock / kWave][2];
    __shared__ float s_acc[kAcc][kBlock];
    __shared__ uint32_t s_lmax;

    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int tile = blockIdx.x;
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int qx = wave & 1, qy = wave >> 1;
    const int pi = tx * kTile + qx * 8 + (lane & 7);
    const int pj = ty * kTile + qy * 8 + (lane >> 3);
    const bool in_img = pi < W && pj < H;
    const float px = (float)pi + 0.5f, py = (float)pj + 0.5f;
    const size_t hw = (size_t)W * H;
    const size_t p = in_img ? (size_t)pj * W + pi : 0;

    float T = in_img ? Tfin[p] : 1.0f;
    const uint32_t L = in_img ? last[p] : 0u;
    const float g0 = in_img ? dL[p] : 0.0f, g1 = in_img ? dL[hw + p] : 0.0f, g2 = in_img ? dL[2 * hw + p] : 0.0f;
    float R0 = op.bg[0], R1 = op.bg[1], R2 = op.bg[2];
    const float amax = op.alpha_max + 0.0f;
    const uint32_t wave_L = (uint32_t)__builtin_amdgcn_readfirstlane((int)wave_max_u32(L));

    if (tid == 0) s_lmax = 0;
#pragma unroll
    for (int k = 0; k < kAcc; ++k) s_acc[k][tid] = 0.0f;
    __syncthreads();
    if (lane == 0) atomicMax(&s_lmax, wave_L);
    __syncthreads();
    const uint32_t lmax = s_lmax;
    const uint32_t start = ranges[tile].x;

    for (int hi = (int)lmax; hi > 0; hi -= kBlock) {
        const int lo = hi > kBlock ? hi - kBlock : 0;
        const int nb = hi - lo;
        uint32_t qm = 0;
        if (tid < nb) {
            const uint32_t g = values[start + (uint32_t)lo + (uint32_t)tid];
            const GaussState s = gs[g];
            const float k2i = s.f1.y * 1.00002f + 1e-5f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int X0i = tx * kTile + (q & 1) * 8, Y0i = ty * kTile + (q >> 1) * 8;
                int X1i = X0i + 8, Y1i = Y0i + 8;
                X1i = X1i > W ? W : X1i;
                Y1i = Y1i > H ? H : Y1i;
                if (X0i < X1i && Y0i < Y1i &&
                    rect_hit(s.f0.x, s.f0.y, s.f0.z, s.f0.w, s.f1.x, k2i, (float)X0i + 0.5f, (float)X1i - 0.5f,
                             (float)Y0i + 0.5f, (float)Y1i - 0.5f))
                    qm |= 1u << q;
            }
            float4 f0, f1;
            float2 f2;
            stage_gauss(s, f0, f1, f2);
            s_f0[tid] = f0;
            s_f1[tid] = f1;
            s_f2[tid] = f2;
            s_id[tid] = g;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint64_t bq = __ballot((qm >> q) & 1u);
            if (lane == 0) {
                s_rel[q][wave][0] = (uint32_t)bq;
                s_rel[q][wave][1] = (uint32_t)(bq >> 32);
            }
        }
        __syncthreads();
        if ((uint32_t)lo < wave_L) {
            for (int wd = kBlock / kWave - 1; wd >= 0; --wd) {
                uint64_t m = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)s_rel[wave][wd][0]) |
                             ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)s_rel[wave][wd][1]) << 32);
                while (m) {
                    const int bit = 63 - __builtin_clzll(m);
                    m &= ~(1ull << bit);
                    const int j = wd * kWave + bit;
                    const uint32_t pos = (uint32_t)(lo + j);
                    if (pos >= wave_L) continue;
                    const float4 f0 = s_f0[j], f1 = s_f1[j];
                    const float2 f2 = s_f2[j];
                    // the forward's exponent and contribution test, bit for bit
                    const float E = exponent_at(f0, row_terms(f0, f1, py), px);
                    const bool c = pos < L && E >= f1.y;
                    if (__ballot(c) == 0) continue;
                    const float dx = px - f0.x, dy = py - f0.y;
                    const float e = __builtin_amdgcn_exp2f(E);
                    const float a = c ? fminf(e, amax) : 0.0f;
                    T = T * __builtin_amdgcn_rcpf(1.0f - a);  // a = 0: T unchanged
                    const float wc = a * T;
                    const float d0 = f1.w - R0, d1 = f2.x - R1, d2 = f2.y - R2;
                    const float ga = T * fmaf(g0, d0, fmaf(g1, d1, g2 * d2));
                    R0 = fmaf(a, d0, R0);
                    R1 = fmaf(a, d1, R1);
                    R2 = fmaf(a, d2, R2);
                    const float wq = (c && e <= amax) ? -0.5f * a * ga : 0.0f;
                    float v[kAcc];
                    v[0] = wq;
                    v[4] = wq * dx;
                    v[5] = wq * dy;
                    v[1] = v[4] * dx;
                    v[2] = v[4] * dy;
                    v[3] = v[5] * dy;
                    v[6] = g0 * wc;
                    v[7] = g1 * wc;
                    v[8] = g2 * wc;
                    wave_sum_to_63(v);
#pragma unroll
                    for (int k = 0; k < kAcc; ++k) {
                        const float r = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[k]), 63));
                        if (lane == k) atomicAdd(&s_acc[k][j], r);
                    }
                }
            }
        }
        __syncthreads();
        if (tid < nb) {
            float v[kAcc];
            bool any = false;
#pragma unroll
            for (int k = 0; k < kAcc; ++k) {
                v[k] = s_acc[k][tid];
                s_acc[k][tid] = 0.0f;
                any |= v[k] != 0.0f;
            }
            if (any) {
                const uint32_t g = s_id[tid];
#pragma unroll
                for (int k = 0; k < kAcc; ++k)
                    if (v[k] != 0.0f) unsafeAtomicAdd(acc + (int64_t)k * acc_stride + g, v[k]);
            }
        }
    }
}

struct DevGrad {
    float *means, *log_scales, *quats, *logits, *sh;
    int64_t stride;
};

__global__ __launch_bounds__(kBlock) void k_preprocess_bwd(DevScene sc, DevCamera cam, DevOptions op, int W, int H,
                                                           const GaussState *__restrict__ gs,
                                                           const float *__restrict__ acc, int64_t acc_stride,
                                                           DevGrad gr) {
    const int64_t st = sc.stride, gst = gr.stride;
    const int nk = (sc.D + 1) * (sc.D + 1);
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < sc.P;
         g += (int64_t)gridDim.x * blockDim.x) {
        float S[kAcc];
        bool any = false;
#pragma unroll
        for (int k = 0; k < kAcc; ++k) {
            S[k] = acc[(int64_t)k * acc_stride + g];
            any |= S[k] != 0.0f;
        }
        if (!any) {
            // culled, or no pixel depends on it
            for (int e = 0; e < 3; ++e) gr.means[e * gst + g] = 0.0f;
            for (int e = 0; e < 3; ++e) gr.log_scales[e * gst + g] = 0.0f;
            for (int e = 0; e < 4; ++e) gr.quats[e * gst + g] = 0.0f;
            gr.logits[g] = 0.0f;
            for (int k = 0; k < 3 * nk; ++k) gr.sh[k * gst + g] = 0.0f;
            continue;
        }
        const GaussState s = gs[g];
        const float A = s.f0.z, B = s.f0.w, C = s.f1.x, o = s.f2.w;
        const float col[3] = {s.f1.w, s.f2.x, s.f2.y};
        // gradients of the blended state
        const float gA = S[1], gB = 2.0f * S[2], gC = S[3];
        const float gu = -2.0f * (A * S[4] + B * S[5]);
        const float gv = -2.0f * (B * S[4] + C * S[5]);
        const float go = -2.0f * S[0] / o;
        float gcol[3];
        for (int ch = 0; ch < 3; ++ch) gcol[ch] = col[ch] > 0.0f ? S[6 + ch] : 0.0f;

        // ---- forward recomputation ----------------------------------------
        const float m[3] = {sc.means[g], sc.means[st + g], sc.means[2 * st + g]};
        const float ls[3] = {sc.log_scales[g], sc.log_scales[st + g], sc.log_scales[2 * st + g]};
        const float qr[4] = {sc.quats[g], sc.quats[st + g], sc.quats[2 * st + g], sc.quats[3 * st + g]};
        const float logit = sc.logits[g];
        const float *Rc = cam.R;
        float t[3];
        for (int r = 0; r < 3; ++r) t[r] = Rc[3 * r] * m[0] + Rc[3 * r + 1] * m[1] + Rc[3 * r + 2] * m[2] + cam.t[r];
        const float sc3[3] = {expf(ls[0]), expf(ls[1]), expf(ls[2])};
        const float qn = sqrtf(qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3]);
        const float w = qr[0] / qn, x = qr[1] / qn, y = qr[2] / qn, z = qr[3] / qn;
        const float iz = 1.0f / t[2];
        const float xt = t[0] * iz, yt = t[1] * iz;
        const float limx = op.jac_clip * (0.5f * (float)W / cam.fx);
        const float limy = op.jac_clip * (0.5f * (float)H / cam.fy);
        const bool clipx = xt < -limx || xt > limx, clipy = yt < -limy || yt > limy;
        const float xc = fminf(fmaxf(xt, -limx), limx), yc = fminf(fmaxf(yt, -limy), limy);
        const float J00 = cam.fx * iz, J02 = -cam.fx * xc * iz, J11 = cam.fy * iz, J12 = -cam.fy * yc * iz;
        const float Rq[9] = {1.0f - 2.0f * (y * y + z * z), 2.0f * (x * y - w * z), 2.0f * (x * z + w * y),
                             2.0f * (x * y + w * z), 1.0f - 2.0f * (x * x + z * z), 2.0f * (y * z - w * x),
                             2.0f * (x * z - w * y), 2.0f * (y * z + w * x), 1.0f - 2.0f * (x * x + y * y)};
        float M[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) M[3 * i + j] = Rq[3 * i + j] * sc3[j];
        float Sig[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                Sig[3 * i + j] = M[3 * i] * M[3 * j] + M[3 * i + 1] * M[3 * j + 1] + M[3 * i + 2] * M[3 * j + 2];
        float Tm[6];
        for (int j = 0; j < 3; ++j) {
            Tm[j] = J00 * Rc[j] + J02 * Rc[6 + j];
            Tm[3 + j] = J11 * Rc[3 + j] + J12 * Rc[6 + j];
        }

        // ---- conic = inverse of X = Sigma' + dilation I: dL/dX = -Y dL/dY Y
        const float hB = 0.5f * gB;
        const float t00 = A * gA + B * hB, t01 = A * hB + B * gC, t10 = B * gA + C * hB, t11 = B * hB + C * gC;
        const float p00 = -(t00 * A + t01 * B), p01 = -(t00 * B + t01 * C);
        const float p10 = -(t10 * A + t11 * B), p11 = -(t10 * B + t11 * C);
        const float gSp[4] = {p00, p01, p10, p11};
        // ---- Sigma' = T Sigma T^T ---------------------------------------------
        // dL/dSigma = T^T gSp T;  dL/dT = (gSp + gSp^T) T Sigma
        float gSig[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                float a = 0.0f;
                for (int u = 0; u < 2; ++u)
                    for (int v = 0; v < 2; ++v) a += Tm[3 * u + i] * gSp[2 * u + v] * Tm[3 * v + j];
                gSig[3 * i + j] = a;
            }
        float TS[6];
        for (int u = 0; u < 2; ++u)
            for (int j = 0; j < 3; ++j)
                TS[3 * u + j] = Tm[3 * u] * Sig[j] + Tm[3 * u + 1] * Sig[3 + j] + Tm[3 * u + 2] * Sig[6 + j];
        const float P2[4] = {2.0f * p00, p01 + p10, p01 + p10, 2.0f * p11};
        float gT[6];
        for (int u = 0; u < 2; ++u)
            for (int j = 0; j < 3; ++j) gT[3 * u + j] = P2[2 * u] * TS[j] + P2[2 * u + 1] * TS[3 + j];
        // ---- T = J R_cam: only J00, J02, J11, J12 vary ------------------------
        const float gJ00 = gT[0] * Rc[0] + gT[1] * Rc[1] + gT[2] * Rc[2];
        const float gJ02 = gT[0] * Rc[6] + gT[1] * Rc[7] + gT[2] * Rc[8];
        const float gJ11 = gT[3] * Rc[3] + gT[4] * Rc[4] + gT[5] * Rc[5];
        const float gJ12 = gT[3] * Rc[6] + gT[4] * Rc[7] + gT[5] * Rc[8];
        // ---- Sigma = M M^T, M = R_q diag(s) ---------------------------------
        float gR[9], gs3[3] = {0.0f, 0.0f, 0.0f};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                float gm = 0.0f;
                for (int l = 0; l < 3; ++l) gm += (gSig[3 * i + l] + gSig[3 * l + i]) * M[3 * l + j];
                gR[3 * i + j] = gm * sc3[j];
                gs3[j] += gm * Rq[3 * i + j];
            }
        for (int j = 0; j < 3; ++j) gr.log_scales[j * gst + g] = gs3[j] * sc3[j];
        // ---- rotation of the unit quaternion, then the normalisation --------
        const float gw = 2.0f * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
        const float gx = 2.0f * (y * gR[1] + z * gR[2] + y * gR[3] - 2.0f * x * gR[4] - w * gR[5] + z * gR[6] +
                                 w * gR[7] - 2.0f * x * gR[8]);
        const float gy = 2.0f * (-2.0f * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] +
                                 z * gR[7] - 2.0f * y * gR[8]);
        const float gz = 2.0f * (-2.0f * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.0f * z * gR[4] +
                                 y * gR[5] + x * gR[6] + y * gR[7]);
        const float dq = w * gw + x * gx + y * gy + z * gz;
        const float iqn = 1.0f / qn;
        gr.quats[g] = (gw - w * dq) * iqn;
        gr.quats[gst + g] = (gx - x * dq) * iqn;
        gr.quats[2 * gst + g] = (gy - y * dq) * iqn;
        gr.quats[3 * gst + g] = (gz - z * dq) * iqn;
        // ---- J and (u, v) from the camera-space mean ----------------------------
        const float iz2 = iz * iz;
        float gt[3] = {0.0f, 0.0f, 0.0f};
        gt[2] += -(gJ00 * cam.fx + gJ11 * cam.fy) * iz2 + (gJ02 * cam.fx * xc + gJ12 * cam.fy * yc) * iz2;
        float gxt = clipx ? 0.0f : -gJ02 * cam.fx * iz;
        float gyt = clipy ? 0.0f : -gJ12 * cam.fy * iz;
        gxt += gu * cam.fx;
        gyt += gv * cam.fy;
        gt[0] += gxt * iz;
        gt[1] += gyt * iz;
        gt[2] -= (gxt * t[0] + gyt * t[1]) * iz2;
        float gm3[3];
        for (int j = 0; j < 3; ++j) gm3[j] = Rc[j] * gt[0] + Rc[3 + j] * gt[1] + Rc[6 + j] * gt[2];
        // ---- opacity ----------------------------------------------------------
        gr.logits[g] = go * o * (1.0f - o);
        // ---- SH colour at the view direction ------------------------------------
        const float dw[3] = {m[0] - cam.eye[0], m[1] - cam.eye[1], m[2] - cam.eye[2]};
        const float dn = sqrtf(dw[0] * dw[0] + dw[1] * dw[1] + dw[2] * dw[2]);
        const float idn = 1.0f / dn;
        const float d[3] = {dw[0] * idn, dw[1] * idn, dw[2] * idn};
        float Y[16], wk[16];
        sh_basis(d[0], d[1], d[2], sc.D, Y);
        for (int k = 0; k < nk; ++k) {
            float a = 0.0f;
            for (int ch = 0; ch < 3; ++ch) {
                gr.sh[(int64_t)(3 * k + ch) * gst + g] = gcol[ch] * Y[k];
                a += gcol[ch] * sc.sh[(int64_t)(3 * k + ch) * st + g];
            }
            wk[k] = a;
        }
        float gd[3];
        sh_basis_grad(d[0], d[1], d[2], sc.D, wk, gd);
        const float dd = d[0] * gd[0] + d[1] * gd[1] + d[2] * gd[2];
        for (int e = 0; e < 3; ++e) gr.means[e * gst + g] = gm3[e] + (gd[e] - d[e] * dd) * idn;
    }
}

}  // namespace

void launch_blend_backward(const GaussState *gs, const uint32_t *values, const uint2 *ranges, const float *Tfin,
                           const uint32_t *last, const float *dL, int W, int H, const DevOptions &op, float *acc,
                           int64_t acc_stride, hipStream_t s) {
    const int tiles_x = (W + kTile - 1) / kTile, tiles_y = (H + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_blend_bwd, dim3((unsigned)(tiles_x * tiles_y)), dim3(kBlock), 0, s, gs, values, ranges,
                       Tfin, last, dL, W, H, tiles_x, op, acc, acc_stride);
}

void launch_preprocess_backward(const DevScene &sc, const DevCamera &cam, const DevOptions &op, int W, int H,
                                const GaussState *gs, const float *acc, int64_t acc_stride, float *g_means,
                                float *g_log_scales, float *g_quats, float *g_logits, float *g_sh,
                                int64_t grad_stride, hipStream_t s) {
    if (sc.P <= 0) return;
    DevGrad gr{g_means, g_log_scales, g_quats, g_logits, g_sh, grad_stride};
    const int64_t blocks = (sc.P + kBlock - 1) / kBlock;
    const unsigned grid = (unsigned)(blocks < 8192 ? blocks : 8192);
    hipLaunchKernelGGL(k_preprocess_bwd, dim3(grid), dim3(kBlock), 0, s, sc, cam, op, W, H, gs, acc, acc_stride, gr);
}

}  // namespace fgs
