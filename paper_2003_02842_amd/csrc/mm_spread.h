// FP32 spreading of one grid tile from per-tap polynomials (Eq. Der:15), shared
// by the tiled spreading kernel (mm_nufft.hip) and the fused small-grid NUFFT
// (mm_fused.hip).  Device code only.
#pragma once
#include <hip/hip_runtime.h>

#include "mm_internal.h"
#include "mm_layout.h"


namespace mm {

// FP32 spreading (Eq. Der:15) from per-tap polynomials, in two phases per chunk
// of staged events:
//   1. each thread evaluates all W taps of its events (tap j is a polynomial in
//      s = f - 1/2 whose coefficients are kernel arguments, so every lane runs the
//      same Horner chains on scalar operands) times the return.  Event i owns a
//      ring of M >= W+1 LDS slots; the tap for cell k goes to slot k mod M and the
//      M - W slots no tap reaches hold 0;
//   2. each thread gathers for its cell pairs (c, c+1), c even: the events with
//      keys c .. c+W (contiguous, sorted) reach cell c at slot c mod M and cell
//      c+1 at the next slot (M even, so the pair is one aligned 8-byte read), and an
//      event that reaches only one of the two cells reads a zero slot for the other.
// No load depends on another, so the gather streams LDS reads.  Cell pairs are the
// real and imaginary parts of one complex grid entry: one float2 store per pair.
//
// spread_tile_poly runs both phases over the events of one tile [a, a + len) of
// one series (rg: the tile's three event ranges, m = -1, 0, 1 periods away) with a
// workgroup of NT threads, leaving cell pair (c, c+1), c = 2 (tid + NT r), in
// acc0[r], acc1[r].  The LDS buffers are the caller's (SpreadLds in mm_layout.h sizes
// them).

// The returns as an array whose type (FP32 or FP64) is known only at run time (one
// uniform branch per load).
struct DpAny {
    using V = double;
    const void* p;
    int f64;
    __device__ V operator[](int64_t i) const
    {
        return f64 ? reinterpret_cast<const double*>(p)[i] : (double)reinterpret_cast<const float*>(p)[i];
    }
};

template <typename Src, int W, int PPT, int NT = 256, int EV = 0>
__device__ __forceinline__ void spread_tile_poly(const double* __restrict__ t, const Src dp, double t0,
                                                 double scale, int Mr, double hw, const PolyParams& pp,
                                                 const int64_t* __restrict__ rg, int a, int len, float* ring,
                                                 unsigned short* keys, unsigned short* first, float (&acc0)[PPT],
                                                 float (&acc1)[PPT])
{
    using L = SpreadLds<W, PPT, NT, EV>;
    constexpr int M = L::M;
    constexpr int EC = L::EC;
    constexpr int SB = EC / NT;
    constexpr int RB = __builtin_ctz(2 * NT);            // log2 of the cells one round covers
    constexpr int DEG = poly_degree_for_width(W);
    int64_t rb[3], nchunk[3];
    int total_chunks = 0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        rb[m] = rg[2 * m];
        const int64_t ne = rg[2 * m + 1] - rb[m];
        nchunk[m] = (ne + EC - 1) / EC;
        total_chunks += (int)nchunk[m];
    }
    auto locate = [&](int q, int64_t& cb, int& n, int& m) {
        m = 0;
        while (q >= nchunk[m]) { q -= (int)nchunk[m]; ++m; }
        cb = rb[m] + (int64_t)q * EC;
        n = (int)min((int64_t)EC, rg[2 * m + 1] - cb);
    };
#pragma unroll
    for (int r = 0; r < PPT; ++r) acc0[r] = acc1[r] = 0.f;
    // leading coefficients of each tap's even and odd Horner chains, held in vector
    // registers for the whole kernel: the first step of a chain then reads one
    // scalar operand instead of two (one scalar operand per instruction)
    float ctop[(W + 1) / 2][2];
#pragma unroll
    for (int j = 0; j < (W + 1) / 2; ++j) {
        ctop[j][0] = pp.c[j][DEG & ~1];
        ctop[j][1] = pp.c[j][(DEG - 1) | 1];
        asm volatile("" : "+v"(ctop[j][0]), "+v"(ctop[j][1]));
    }
    // Chunk staging runs two chunks ahead: two register sets alternate, so that the
    // loads of chunk q+1 are already in flight while chunk q is staged, and those of
    // chunk q+2 are issued as soon as chunk q's registers are free.
    // The loads are unconditional (past the end of a chunk, or past the last chunk,
    // they repeat its last event), so every path issues the same loads and the
    // compiler's wait before staging a chunk leaves the other set in flight.
    using DPT = typename Src::V;
    auto load_chunk = [&](int qq, double (&tvx)[SB], DPT (&dvx)[SB]) {
        int64_t cb2; int n2, m2;
        locate(min(qq, total_chunks - 1), cb2, n2, m2);
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int64_t ii = cb2 + min((int)threadIdx.x + NT * u, n2 - 1);
            tvx[u] = t[ii];
            dvx[u] = dp[ii];
        }
    };
    auto chunk = [&](int q, double (&tv)[SB], DPT (&dv)[SB]) {
        int64_t cb; int n, m;
        locate(q, cb, n, m);
        // key = first-tap cell - (a + (m - 1) Mr) + W - 1, the first-tap cell being floor(g - hw) + 1
        const int kofs = (int)((int64_t)W - (int64_t)a - (int64_t)(m - 1) * Mr);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int i = (int)threadIdx.x + NT * u;
            if (i < n) {
                // cell_of<false> with the cell in 32 bits (|floor(g - hw)| < Mr + w < 2^31)
                const double tt = fma(__dsub_rn(tv[u], t0), scale, -hw);
                const double fl = floor(tt);
                const double f = __dsub_rn(tt, fl);
                const int key = (int)fl + kofs;              // >= 0; tap j reaches cell key - W + 1 + j
                const float sv = (float)(f - 0.5);
                const float v = (float)dv[u];
                // tap j = v (E_j(s^2) + s O_j(s^2)) and, by the kernel's symmetry, tap W-1-j =
                // v (E_j(s^2) - s O_j(s^2)): even and odd coefficients by Horner in s^2,
                // the return folded in as v E_j and (v s) O_j
                const float s2 = sv * sv, vs = v * sv;
                float tap[W];
#pragma unroll
                for (int j = 0; j < (W + 1) / 2; ++j) {
                    constexpr int DE = DEG & ~1, DO = (DEG - 1) | 1;   // top even and odd powers
                    float ev = fmaf(ctop[j][0], s2, pp.c[j][DE - 2]), od = fmaf(ctop[j][1], s2, pp.c[j][DO - 2]);
#pragma unroll
                    for (int k = DE - 4; k >= 0; k -= 2) ev = fmaf(ev, s2, pp.c[j][k]);
#pragma unroll
                    for (int k = DO - 4; k >= 1; k -= 2) od = fmaf(od, s2, pp.c[j][k]);
                    const float vev = v * ev;
                    tap[j] = fmaf(vs, od, vev);
                    if (W - 1 - j != j) tap[W - 1 - j] = fmaf(-vs, od, vev);
                }
                // slot of tap j: base + j, or base + j - M past the end of the ring; each
                // store picks one of two row pointers and adds j as a constant offset
                const int base = (key - W + 1 + M) % M;     // slot of tap 0: (key - W + 1) mod M, key >= 0
                const int r1 = 4 * (i * M + base), r2 = r1 - 4 * M;   // byte offsets of the two rows
                char* const rb = reinterpret_cast<char*>(ring);
#pragma unroll
                for (int j = 0; j < M; ++j)
                    *reinterpret_cast<float*>(rb + (j < M - base ? r1 : r2) + 4 * j) = j < W ? tap[j] : 0.f;
                keys[i] = (unsigned short)key;
            }
        }
        // this register set is free again: load the chunk after next into it
        load_chunk(q + 2, tv, dv);
        __syncthreads();
        // the chunk's key range, the same for every lane: held in scalar registers
        const int kmin = __builtin_amdgcn_readfirstlane(keys[0]);
        const int kmax = __builtin_amdgcn_readfirstlane(keys[n - 1]);
        for (int i = 1 + threadIdx.x; i < n; i += NT) {
            const int k1 = keys[i];
            for (int k = keys[i - 1] + 1; k <= k1; ++k) first[k] = (unsigned short)i;
        }
        __syncthreads();
        // rounds whose cell pairs (c, c+1), c = 2 (tid + NT r), can meet the chunk:
        // kmin - W <= c <= kmax; the others are skipped by a scalar branch
        const int r_lo = max(kmin - W, 0) >> RB, r_hi = kmax >> RB;
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
            if (r < r_lo || r > r_hi) continue;
            const int c = 2 * ((int)threadIdx.x + NT * r);
            if (c >= len || c + W < kmin || c > kmax) continue;
            const int lo = (c <= kmin) ? 0 : first[c];
            const int hi = (c + W + 1 > kmax) ? n : first[c + W + 1];
            const float2* rp = reinterpret_cast<const float2*>(ring + (c % M)) + (lo * M) / 2;
            float s0 = 0.f, s1 = 0.f, u0 = 0.f, u1 = 0.f, p0 = 0.f, p1 = 0.f, q0 = 0.f, q1 = 0.f;
            int e = lo;
            for (; e + 3 < hi; e += 4, rp += 2 * M) {
                const float2 x = rp[0], y = rp[M / 2], z = rp[M], zz = rp[3 * M / 2];
                s0 += x.x;
                s1 += x.y;
                u0 += y.x;
                u1 += y.y;
                p0 += z.x;
                p1 += z.y;
                q0 += zz.x;
                q1 += zz.y;
            }
            for (; e < hi; ++e, rp += M / 2) {
                const float2 x = rp[0];
                s0 += x.x;
                s1 += x.y;
            }
            acc0[r] += (s0 + u0) + (p0 + q0);
            acc1[r] += (s1 + u1) + (p1 + q1);
        }
        };
    double tva[SB], tvb[SB];
    DPT dva[SB], dvb[SB];
    if (total_chunks > 0) {
        load_chunk(0, tva, dva);
        load_chunk(1, tvb, dvb);
    }
    for (int q = 0; q < total_chunks; q += 2) {
        chunk(q, tva, dva);
        if (q + 1 >= total_chunks) break;
        chunk(q + 1, tvb, dvb);
    }
}


}  // namespace mm
