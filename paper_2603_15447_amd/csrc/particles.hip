// Particle ring (Sec. 5's particle test): particles move along a closed ring
// of chained cubic Bezier segments; every frame a particle advances its
// phase, evaluates its position on the ring and hands it to a consumer, a
// K-step arithmetic recurrence standing in for the shader's other work, so
// the frame can be made as compute-bound as wanted.  The position comes from
// one of four ring representations (what the paper compares: shader
// arithmetic against reads of small textures):
//   0 polynomial: control points seg[N][3][4], Bernstein form;
//   1 Seiler terms [N][3][4] (bz_bezier_to_seiler): three lerps;
//   2 Seiler textures [N][3][4] (bz_build_texture, Seiler): the emulated
//     8-bit filter read at (t, st);
//   3 sampled table [3][N*S] (bz_particle_ring_table: segment k at t = j/S,
//     de Casteljau): one lerp between neighbouring samples.
#include "curves_impl.h"
#include "texfilter.h"

namespace bzi {
namespace {

struct ParticleArgs {
    const float *ring;
    uint32_t n_seg, samples;  // samples: table method only
    float *T;
    const float *speed;
    float dt;
    uint32_t np;
    int iters;
    float *pos;               // [3][np]
    float *shade;             // [np]
};

template <int METHOD>
__global__ __launch_bounds__(kBlock) void k_particles(ParticleArgs a) {
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= a.np) return;
    const float nf = static_cast<float>(a.n_seg);
    float Tn;
    {
#pragma clang fp contract(off)
        Tn = a.T[p] + a.speed[p] * a.dt;
        if (Tn >= nf) Tn -= nf;
        if (Tn < 0.0f) Tn += nf;
        if (Tn >= nf) Tn = 0.0f;  // only if the subtraction rounded up to N
    }
    const float kf = __builtin_fminf(__builtin_floorf(Tn), static_cast<float>(a.n_seg - 1));
    const uint32_t k = min(static_cast<uint32_t>(__builtin_fmaxf(kf, 0.0f)), a.n_seg - 1);  // NaN -> 0
    const float t = Tn - static_cast<float>(k);
    float xyz[3];
    if constexpr (METHOD == 3) {
        const uint32_t ntab = a.n_seg * a.samples;
        float x, f;
        uint32_t i;
        {
#pragma clang fp contract(off)
            x = Tn * static_cast<float>(a.samples);
            const float fi = __builtin_fminf(__builtin_floorf(x), static_cast<float>(ntab - 1));
            i = min(static_cast<uint32_t>(__builtin_fmaxf(fi, 0.0f)), ntab - 1);
            f = x - static_cast<float>(i);
        }
        const uint32_t i1 = i + 1 == ntab ? 0 : i + 1;
#pragma unroll
        for (int c = 0; c < 3; ++c) xyz[c] = lerp(a.ring[c * ntab + i], a.ring[c * ntab + i1], f);
    } else {
        const float4 *__restrict__ r4 = reinterpret_cast<const float4 *>(a.ring) + static_cast<size_t>(k) * 3;
        float st = 0.0f, wt = 0.0f, wst = 0.0f;
        float B[4];
        if constexpr (METHOD == 0) bernstein_basis<3>(t, B);
        if constexpr (METHOD == 1 || METHOD == 2) {
#pragma clang fp contract(off)
            st = (1.0f - t) * t;
        }
        if constexpr (METHOD == 2) {
            wt = tx_axis_weight(t, 8, 0);
            wst = tx_axis_weight(st, 8, 0);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float4 q = r4[c];
            const float v[4] = {q.x, q.y, q.z, q.w};
            if constexpr (METHOD == 0) {
                xyz[c] = dot_basis<3>(B, v);
            } else if constexpr (METHOD == 1) {
                xyz[c] = eval_seiler<3>(v, t, st);
            } else {
                xyz[c] = tx_bilinear(v, wt, wst);
            }
        }
    }
    // consumer: v <- a v + (b x + c y + d z), K times
    const float drive = __builtin_fmaf(0.0625f, xyz[2], __builtin_fmaf(-0.125f, xyz[1], 0.25f * xyz[0]));
    float v = 0.0f;
#pragma unroll 4
    for (int i = 0; i < a.iters; ++i) v = __builtin_fmaf(0.71875f, v, drive);
    a.T[p] = Tn;
#pragma unroll
    for (int c = 0; c < 3; ++c) st_stream(a.pos + static_cast<size_t>(c) * a.np + p, xyz[c]);
    st_stream(a.shade + p, v);
}

// Table of the ring for method 3: one thread per (segment, sample).
__global__ __launch_bounds__(kBlock) void k_ring_table(const float *__restrict__ ring, uint32_t n_seg,
                                                       uint32_t samples, float *__restrict__ table) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t n = n_seg * samples;
    if (i >= n) return;
    const uint32_t k = i / samples, j = i - k * samples;
    const float t = static_cast<float>(j) / static_cast<float>(samples);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float b[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) b[e] = ring[(static_cast<size_t>(k) * 3 + c) * 4 + e];
        table[static_cast<size_t>(c) * n + i] = eval_dc<3>(b, t);
    }
}

}  // namespace
}  // namespace bzi

using namespace bzi;

extern "C" int bz_particle_ring_table(const float *ring, int64_t n_seg, int samples, float *table, bz_stream stream) {
    return guarded("bz_particle_ring_table", [&]() -> int {
        const char *fn = "bz_particle_ring_table";
        if (n_seg < 1 || n_seg > (int64_t(1) << 20)) return fail(BZ_ERR_SHAPE, "%s: n_seg not in 1..2^20", fn);
        if (samples < 1 || n_seg * samples > (int64_t(1) << 24))
            return fail(BZ_ERR_SHAPE, "%s: samples (n_seg*samples at most 2^24)", fn);
        if (!ring || !table) return fail(BZ_ERR_NULL, "%s: ring and table are required", fn);
        if (!aligned(ring, 4) || !aligned(table, 4)) return fail(BZ_ERR_ALIGN, "%s: misaligned", fn);
        const uint32_t n = static_cast<uint32_t>(n_seg * samples);
        hipLaunchKernelGGL(bzi::k_ring_table, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, as_stream(stream), ring,
                           static_cast<uint32_t>(n_seg), static_cast<uint32_t>(samples), table);
        BZ_CHECK_LAUNCH("k_ring_table");
        return BZ_OK;
    });
}

extern "C" int bz_particles_step(int method, const float *ring, int64_t n_seg, int samples, float *T,
                                 const float *speed, float dt, int64_t n_particles, int iters, float *pos,
                                 float *shade, bz_stream stream) {
    return guarded("bz_particles_step", [&]() -> int {
        const char *fn = "bz_particles_step";
        if (method < 0 || method > 3) return fail(BZ_ERR_UNSUPPORTED, "%s: method %d", fn, method);
        if (n_seg < 1 || n_seg > (int64_t(1) << 20)) return fail(BZ_ERR_SHAPE, "%s: n_seg not in 1..2^20", fn);
        if (method == 3 && (samples < 1 || n_seg * samples > (int64_t(1) << 24)))
            return fail(BZ_ERR_SHAPE, "%s: samples (n_seg*samples at most 2^24)", fn);
        if (n_particles < 0 || n_particles > (int64_t(1) << 31)) return fail(BZ_ERR_SHAPE, "%s: n_particles", fn);
        if (iters < 0) return fail(BZ_ERR_SHAPE, "%s: iters", fn);
        if (n_particles == 0) return BZ_OK;
        if (!ring || !T || !speed || !pos || !shade) return fail(BZ_ERR_NULL, "%s: all arrays are required", fn);
        if (!aligned(ring, 16) || !aligned(T, 4) || !aligned(speed, 4) || !aligned(pos, 4) || !aligned(shade, 4))
            return fail(BZ_ERR_ALIGN, "%s: ring needs 16-byte alignment", fn);
        ParticleArgs a;
        a.ring = ring;
        a.n_seg = static_cast<uint32_t>(n_seg);
        a.samples = static_cast<uint32_t>(method == 3 ? samples : 1);
        a.T = T;
        a.speed = speed;
        a.dt = dt;
        a.np = static_cast<uint32_t>(n_particles);
        a.iters = iters;
        a.pos = pos;
        a.shade = shade;
        const uint32_t blocks = static_cast<uint32_t>((n_particles + kBlock - 1) / kBlock);
        const hipStream_t s = as_stream(stream);
        switch (method) {
            case 0: hipLaunchKernelGGL(k_particles<0>, dim3(blocks), dim3(kBlock), 0, s, a); break;
            case 1: hipLaunchKernelGGL(k_particles<1>, dim3(blocks), dim3(kBlock), 0, s, a); break;
            case 2: hipLaunchKernelGGL(k_particles<2>, dim3(blocks), dim3(kBlock), 0, s, a); break;
            default: hipLaunchKernelGGL(k_particles<3>, dim3(blocks), dim3(kBlock), 0, s, a); break;
        }
        BZ_CHECK_LAUNCH("k_particles");
        return BZ_OK;
    });
}
