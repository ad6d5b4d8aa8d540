// The enumeration kernel template (instantiated in enum_q8_*.hip).
#pragma once

#include "kernels_q8.h"
#include "enum_common.h"

namespace ibmc {

// ---- register-level helpers (gfx950) -------------------------------------

typedef short short2_t __attribute__((ext_vector_type(2)));

// Requantise four accumulators: t = clamp(acc >> s, lo, hi), packed as the
// four low bytes.  With (lo, hi) = (-64, 63) and acc = u - 64 * 2^s this is
// the offset activation a - 64 of a = clamp(floor(u / 2^s), 0, 127); with
// (lo, hi) = (0, 127) and acc = u it is a itself.  (Plain code on purpose:
// the compiler then sees every register dependence, including the wait
// states that reading MFMA results requires.)
__device__ __forceinline__ int requant4_clamp(v4i acc, int s, int lo, int hi) {
    int t[4];
#pragma unroll
    for (int z = 0; z < 4; ++z) t[z] = min(max(acc[z] >> s, lo), hi);
    const unsigned l2 = __builtin_amdgcn_perm((unsigned)t[1], (unsigned)t[0], 0x0c0c0400u);
    const unsigned h2 = __builtin_amdgcn_perm((unsigned)t[3], (unsigned)t[2], 0x04000c0cu);
    return (int)(l2 | h2);
}

__device__ __forceinline__ int requant4_offset(v4i acc, int s) { return requant4_clamp(acc, s, -64, 63); }

// Fast hidden epilogue: the accumulator is alpha * u - 32768 with
// alpha * 2^s = 256.  Saturated to int16 (two values per conversion) and
// capped at -1, byte 1 of each half is a - 128 for a = clamp(floor(u / 2^s),
// 0, 127): below u = 0 the conversion saturates to -32768 (byte -128), from
// a = 128 on the cap gives byte -1.
__device__ __forceinline__ int requant4_sat(v4i acc) {
    const short2_t m1 = {(short)-1, (short)-1};
    const short2_t p0 = __builtin_elementwise_min(__builtin_amdgcn_cvt_pk_i16(acc[0], acc[1]), m1);
    const short2_t p1 = __builtin_elementwise_min(__builtin_amdgcn_cvt_pk_i16(acc[2], acc[3]), m1);
    return (int)__builtin_amdgcn_perm(__builtin_bit_cast(unsigned, p1), __builtin_bit_cast(unsigned, p0),
                                      0x07050301u);
}

// a - 64 bytes -> 2 (a - 64) bytes (still int8: [-128, 126]); the bit that
// crosses into the next byte is masked off.
__device__ __forceinline__ int double_bytes(int d) { return (int)(((unsigned)d << 1) & 0xfefefefeu); }

__device__ __forceinline__ int as_int(short2_t v) { return __builtin_bit_cast(int, v); }
__device__ __forceinline__ short2_t as_s2(int v) { return __builtin_bit_cast(short2_t, v); }

// Base of the current segment: clean first-layer potentials plus the
// prefix's column updates e * W1[:, p], one position per lane and K-block
// (positions lane + 64 r, coalesced).  Packed path: int16 v = f u - 16384
// into the wave's LDS slice base16, clamped so that adding any last-element
// update cannot overflow; int32 path: u - 64 * 2^s into base32.
template <int KB1>
__device__ __forceinline__ void build_base(const Cursor &c, const EnumParams &P, const int32_t *u0s, int32_t *base32,
                                           int16_t *base16, int lane, int ulo, int uhi) {
    const int H1 = KB1 * 64;
    int pp[kMaxK], ee[kMaxK];
    int np = 0;
    if (c.mode == SEG_PLAIN) {
        np = c.k - 1;
#pragma unroll
        for (int j = 0; j < kMaxK; ++j) {
            pp[j] = 0;
            ee[j] = 0;
            if (j < np) {
                pp[j] = c.pre[j];
                const int xv = wave_uniform((int)gld(c.img + pp[j]));
                ee[j] = clamp_pixel(xv + wave_uniform((int)gld(c.dl + c.dg[j]))) - xv;
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < kMaxK; ++j) { pp[j] = 0; ee[j] = 0; }
        if (c.mode == SEG_SHELL) {
            np = 1;
            const int head = wave_uniform(gld(P.jobs[c.job].order + c.shell));
            pp[0] = head / c.m;
            const int xv = wave_uniform((int)gld(c.img + pp[0]));
            ee[0] = clamp_pixel(xv + wave_uniform((int)gld(c.dl + head - pp[0] * c.m))) - xv;
        }
    }
    const int off = 64 << P.net.shift[0];
    const int f = P.net.f1;
#pragma unroll
    for (int r = 0; r < KB1; ++r) {
        const int q = lane + 64 * r;
        int v = u0s[q];
        for (int j = 0; j < np; ++j) v += ee[j] * (int)P.net.W1T[(int64_t)pp[j] * H1 + q];
        if (P.packed) {
            // u is first clamped to [ulo, uhi], outside of which the product
            // clamps to the same bound, so that f u fits in 32 bits
            const int w = min(max(v, ulo), uhi) * f - 16384;
            base16[q] = (int16_t)min(max(w, P.vb_lo), P.vb_hi);
        } else {
            base32[q] = v - off;
        }
    }
}

// Rank of a recorded point (see the header's point rank) from the segment's
// uniform part: plain segments and single-pixel lists add p m^k + i to r0;
// level-2 shells combine the head (ph, ih) and the partner (p, i) in pixel
// order.
struct EmitInfo {
    int prop, k, slot, mode, n, m, ph, ih;
    int64_t r0, mk;
};

template <class PT>
__device__ __forceinline__ EmitInfo make_emit_info(const Cursor &c, const PT &P) {
    EmitInfo e;
    e.prop = c.prop;
    e.k = c.k;
    e.slot = c.slot;
    e.mode = c.mode;
    e.n = c.n;
    e.m = c.m;
    e.ph = 0;
    e.ih = 0;
    int64_t mk = 1;
    for (int j = 0; j < c.k; ++j) mk *= c.m;
    e.mk = mk;
    if (c.mode == SEG_SHELL) {
        const int head = wave_uniform(gld(P.jobs[c.job].order + c.shell));
        e.ph = head / c.m;
        e.ih = head - e.ph * c.m;
        e.r0 = 0;
        return e;
    }
    // plain k >= 1 (and single-pixel lists, k == 1): prefix pixels pre[0..k-2]
    int64_t s = 0, d = 0;
    if (c.mode == SEG_PLAIN) {
        // fixed trip count: the cursor's arrays stay in registers
#pragma unroll
        for (int j = 0; j < kMaxK; ++j) {
            if (j < c.k - 1) {
                s += binom_small(c.n - 1 - c.pre[j], c.k - j);
                d = d * c.m + c.dg[j];
            }
        }
    }
    e.r0 = (binom_small(c.n, c.k) - 1 - s - (c.n - 1)) * mk + d * c.m;
    return e;
}

__device__ __forceinline__ int64_t rank_of(const EmitInfo &e, int p, int i) {
    if (e.mode != SEG_SHELL) return e.r0 + (int64_t)p * e.mk + i;
    const bool hf = e.ph < p;
    const int a = hf ? e.ph : p, b = hf ? p : e.ph;
    const int da = hf ? e.ih : i, db = hf ? i : e.ih;
    const int64_t x = e.n - 1 - a;
    const int64_t c2n = (int64_t)e.n * (e.n - 1) / 2;
    return (c2n - 1 - x * (x - 1) / 2 - (e.n - 1 - b)) * e.mk + (int64_t)da * e.m + db;
}

// Emission state of a chunk as lanes of one VGPR (wave-uniform values, read
// back only when a tile records violations): lanes w and 4 + w hold the low
// and high half of segment w's rank offset, the others the fields below.
enum : int {
    EI_PROP = 8, EI_K, EI_SLOT, EI_MODE, EI_N, EI_M, EI_PH, EI_IH, EI_MKLO, EI_MKHI, EI_GCLO, EI_GCHI
};
static_assert(kSegGroup <= 4, "rank offsets take lanes 0..7");

__device__ __forceinline__ int lane_put(int v, int idx, int x) { return (int)__lane_id() == idx ? x : v; }
__device__ __forceinline__ int lane_get(int v, int idx) { return __builtin_amdgcn_readlane(v, idx); }

// Segment w's emission info into v (the group's common fields with w == 0).
__device__ __forceinline__ int einfo_pack(const EmitInfo &e, int w, int v) {
    v = lane_put(v, w, (int)(uint32_t)e.r0);
    v = lane_put(v, 4 + w, (int)(e.r0 >> 32));
    if (w == 0) {
        v = lane_put(v, EI_PROP, e.prop);
        v = lane_put(v, EI_K, e.k);
        v = lane_put(v, EI_SLOT, e.slot);
        v = lane_put(v, EI_MODE, e.mode);
        v = lane_put(v, EI_N, e.n);
        v = lane_put(v, EI_M, e.m);
        v = lane_put(v, EI_PH, e.ph);
        v = lane_put(v, EI_IH, e.ih);
        v = lane_put(v, EI_MKLO, (int)(uint32_t)e.mk);
        v = lane_put(v, EI_MKHI, (int)(e.mk >> 32));
    }
    return v;
}

__device__ __forceinline__ int64_t lane_get64(int v, int lo, int hi) {
    return (int64_t)(((uint64_t)(uint32_t)lane_get(v, hi) << 32) | (uint32_t)lane_get(v, lo));
}

__device__ __forceinline__ EmitInfo einfo_unpack(int v, int w) {
    EmitInfo e;
    e.prop = lane_get(v, EI_PROP);
    e.k = lane_get(v, EI_K);
    e.slot = lane_get(v, EI_SLOT);
    e.mode = lane_get(v, EI_MODE);
    e.n = lane_get(v, EI_N);
    e.m = lane_get(v, EI_M);
    e.ph = lane_get(v, EI_PH);
    e.ih = lane_get(v, EI_IH);
    e.mk = lane_get64(v, EI_MKLO, EI_MKHI);
    e.r0 = lane_get64(v, w, 4 + w);
    return e;
}

// Cross-row exchange without LDS: v_permlane32_swap / v_permlane16_swap of
// a value with itself give, in every lane, the pair (lower-half value,
// upper-half value) of lanes l and l ^ 32, resp. (even-row value, odd-row
// value) of lanes l and l ^ 16 (rows: 16 lanes).
struct LanePair {
    int lo, hi;
};
__device__ __forceinline__ LanePair swap32(int x) {
    const auto p = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return LanePair{(int)p[0], (int)p[1]};
}
__device__ __forceinline__ LanePair swap16(int x) {
    const auto p = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return LanePair{(int)p[0], (int)p[1]};
}

// Row G's value (lane 16 G + l % 16) in every lane; G wave-uniform.
__device__ __forceinline__ int row_bcast(int x, int G) {
    const LanePair a = swap32(x);
    const LanePair b = swap16(G >= 2 ? a.hi : a.lo);
    return (G & 1) ? b.hi : b.lo;
}

// Lowest-index maximum over one 16-row tile of logits (this lane's four
// rows, classes 16 mt + 4 g + t), combined into (value, index, count).
// CHECK: skip classes >= ncls (else their logits are INT32_MIN, below any
// real logit, which the int32 headroom check keeps above INT32_MIN).
template <bool CHECK>
__device__ __forceinline__ void argmax_tile(v4i acc, int mt, int g, int ncls, int &bv, int &bi, int &bc) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int cls = mt * 16 + g * 4 + t;
        const int v = acc[t];
        if (!CHECK || cls < ncls) {
            if (v > bv) { bv = v; bi = cls; bc = 1; }
            else if (v == bv) { bc += 1; bi = min(bi, cls); }
        }
    }
}

// Combine the four lane groups holding the same point (both lanes of a
// pair reach the same, symmetric, result).
__device__ __forceinline__ void argmax_pair(const LanePair &v, const LanePair &i, const LanePair &c, int &bv, int &bi,
                                            int &bc) {
    if (v.lo > v.hi) { bv = v.lo; bi = i.lo; bc = c.lo; }
    else if (v.hi > v.lo) { bv = v.hi; bi = i.hi; bc = c.hi; }
    else { bv = v.lo; bi = min(i.lo, i.hi); bc = c.lo + c.hi; }
}
__device__ __forceinline__ void argmax_combine(int &bv, int &bi, int &bc) {
    argmax_pair(swap16(bv), swap16(bi), swap16(bc), bv, bi, bc);
    argmax_pair(swap32(bv), swap32(bi), swap32(bc), bv, bi, bc);
}

// Per-wave record output: slots come in blocks of kRecBlock from one atomic
// (most tiles then write without any atomic), and counterexample / tie
// counts gather per level slot until the slot changes.  All fields are
// wave-uniform.
struct RecOut {
    int64_t next, end;   // free slots of the current block
    int slot;            // level slot being counted
    bool notified;       // this wave has reported its first counterexample
    unsigned long long cex, ties;
};

__device__ __forceinline__ void rec_flush_counts(RecOut &o, int lane) {
    if (o.slot >= 0 && lane == 0) {
        const EnumParams &P = cold_params<EnumParams>();
        if (o.cex) atomicAdd(P.slot_cex + o.slot, o.cex);
        if (o.ties) atomicAdd(P.slot_ties + o.slot, o.ties);
    }
    o.cex = 0;
    o.ties = 0;
}

__device__ __forceinline__ void rec_tally(RecOut &o, int slot, unsigned ncex, unsigned nties, int lane) {
    if (slot != o.slot) {
        rec_flush_counts(o, lane);
        o.slot = slot;
    }
    o.cex += ncex;
    o.ties += nties;
}

// At the wave's end: counts out, sentinels into the block's unused slots.
__device__ __forceinline__ void rec_finish(RecOut &o, int lane) {
    rec_flush_counts(o, lane);
    const EnumParams &P = cold_params<EnumParams>();
    const int64_t idx = o.next + lane;
    if (lane < kRecBlock && idx < o.end && idx < P.rec_cap) {
        DevRec r;
        r.rank = -1;
        r.prop = -1;
        r.klab = 0;
        P.recs[idx] = r;
    }
}

// Record the violations of segment w's NT 16-point tiles (lanes of group 0
// carry the points) in the wave's current block, continuing in a new block
// when it runs out (the tiles hold at most 16 NT <= kRecBlock records, so one
// new block always suffices).  The emission info and the parameter block are
// read once for all tiles.  einfo: the chunk's packed emission info.
template <int NT>
__device__ __forceinline__ void emit_tiles(RecOut &o, int einfo, int w, const bool (&viol)[NT], const int (&p)[NT],
                                           const int (&i)[NT], const int (&label)[NT], int lane) {
    static_assert(16 * NT <= kRecBlock, "one block reservation per call");
    unsigned long long vm[NT];
    int n = 0;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        vm[nt] = __ballot(viol[nt]);
        n += __popcll(vm[nt]);
    }
    if (!n) return;
    const EnumParams &P = cold_params<EnumParams>();
    const EmitInfo e = einfo_unpack(einfo, w);
    const int64_t room = o.end - o.next;
    int64_t nb = 0;
    if (n > room) {
        unsigned long long start = 0;
        if (lane == 0) start = atomicAdd(P.rec_count, (unsigned long long)kRecBlock);
        nb = (int64_t)wave_uniform(start);  // lane 0's value
    }
    // side effects of a counterexample, once per wave: its chunks come in
    // increasing order, so the first one holds the wave's smallest chunk
    if (P.notify && !o.notified) {
        o.notified = true;
        const int64_t gchunk = lane_get64(einfo, EI_GCLO, EI_GCHI);
        if (lane == 0) {
            // the host-mapped hit flag is written once per grid, by the wave
            // that lowers first_chunk from its initial value (a write per
            // wave would keep the bus and the host's polled line busy)
            const unsigned long long was =
                P.track_first ? atomicMin(P.first_chunk, (unsigned long long)gchunk) : 0ull;
            if (P.hit_host && was == ~0ull) *P.hit_host = 1;
            if (P.stop_on_first) *P.stop_flag = 1;
        }
    }
    rec_tally(o, e.slot, (unsigned)n, 0u, lane);
    const unsigned long long below = (1ull << lane) - 1ull;
    int before = 0;  // records of the earlier tiles
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        if (viol[nt]) {
            const int t = before + __popcll(vm[nt] & below);
            const int64_t idx = t < room ? o.next + t : nb + (t - room);
            if (idx < P.rec_cap) {
                DevRec r;
                r.rank = rank_of(e, p[nt], i[nt]);
                r.prop = e.prop;
                r.klab = (e.k << 24) | (label[nt] & 0xffffff);
                P.recs[idx] = r;
            }
        }
        before += __popcll(vm[nt]);
    }
    if (n > room) {
        o.next = nb + (n - room);
        o.end = nb + kRecBlock;
    } else {
        o.next += n;
    }
}

__device__ __forceinline__ unsigned fold_groups(unsigned long long m) {
    return (unsigned)((m | (m >> 16) | (m >> 32) | (m >> 48)) & 0xffffull);
}

// Loads of one chunk's first layer, issued together (a chunk ahead of
// their use): each tile's pixel, delta and weight column slice (packed path:
// 16 int16 of f W1 per K-block in two 16-byte halves; int32 path: 16 int8 of
// W1, the second half then repeats the first).  The path is a uniform
// select, so that no branch separates the loads from each other.
template <int KB1, int NT>
struct L1Loads {
    int xv[NT], dv[NT];
    v4i wa[NT][KB1], wb[NT][KB1];
};

template <int KB1, int NT>
__device__ __forceinline__ void layer1_issue(const Cursor &c, const QNetDev &net, bool packed, const int (&plast)[NT],
                                             const int (&ilast)[NT], int g, L1Loads<KB1, NT> &ld) {
    constexpr int H1 = KB1 * 64;
    const int kstride = packed ? 128 : 64;  // bytes per K-block of a column
    const int boff = packed ? 16 : 0;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        ld.xv[nt] = gld(c.img + plast[nt]);
        ld.dv[nt] = gld(c.dl + ilast[nt]);
        const char *wp = packed ? reinterpret_cast<const char *>(net.W1T16 + plast[nt] * H1 + g * 16)
                                : reinterpret_cast<const char *>(net.W1T + plast[nt] * H1 + g * 16);
#pragma unroll
        for (int kb = 0; kb < KB1; ++kb) {
            ld.wa[nt][kb] = gld(reinterpret_cast<const v4i *>(wp + kb * kstride));
            ld.wb[nt][kb] = gld(reinterpret_cast<const v4i *>(wp + kb * kstride + boff));
        }
    }
}

// First layer, packed int16 path: u = base + e W1[:, p] as v = f u - 16384
// in 16-bit halves, clamped to [-16384, 16383], whose byte 1 is a - 64.  The
// base of this lane group's 16 positions per K-block comes from LDS.
// DBL: bytes 2 (a - 64) instead, from the saturated sum v + v (its byte 1 is
// floor(v / 128), 2 (a - 64) plus a low bit that is masked off); the
// pre-clamped base keeps v itself inside int16.
template <int KB1, int NT, bool DBL>
__device__ __forceinline__ void layer1_packed(const L1Loads<KB1, NT> &ld, const int (&ev)[NT], const int16_t *base16,
                                              int g, v4i (&a1)[NT][KB1]) {
    const short2_t vlo = {(short)-16384, (short)-16384};
    const short2_t vhi = {(short)16383, (short)16383};
    v4i bl[KB1], bh[KB1];
#pragma unroll
    for (int kb = 0; kb < KB1; ++kb) {
        bl[kb] = *reinterpret_cast<const v4i *>(base16 + kb * 64 + g * 16);
        bh[kb] = *reinterpret_cast<const v4i *>(base16 + kb * 64 + g * 16 + 8);
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const short2_t e2 = {(short)ev[nt], (short)ev[nt]};
#pragma unroll
        for (int kb = 0; kb < KB1; ++kb) {
            const int wv[8] = {ld.wa[nt][kb][0], ld.wa[nt][kb][1], ld.wa[nt][kb][2], ld.wa[nt][kb][3],
                               ld.wb[nt][kb][0], ld.wb[nt][kb][1], ld.wb[nt][kb][2], ld.wb[nt][kb][3]};
            const int bv[8] = {bl[kb][0], bl[kb][1], bl[kb][2], bl[kb][3], bh[kb][0], bh[kb][1], bh[kb][2], bh[kb][3]};
            int pr2[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                short2_t u = as_s2(bv[t]) + e2 * as_s2(wv[t]);
                if constexpr (DBL) {
                    u = __builtin_elementwise_add_sat(u, u);
                } else {
                    u = __builtin_elementwise_max(u, vlo);
                    u = __builtin_elementwise_min(u, vhi);
                }
                pr2[t] = as_int(u);
            }
            const unsigned msk = DBL ? 0xfefefefeu : 0xffffffffu;
            a1[nt][kb] = v4i{(int)(__builtin_amdgcn_perm(pr2[1], pr2[0], 0x07050301u) & msk),
                             (int)(__builtin_amdgcn_perm(pr2[3], pr2[2], 0x07050301u) & msk),
                             (int)(__builtin_amdgcn_perm(pr2[5], pr2[4], 0x07050301u) & msk),
                             (int)(__builtin_amdgcn_perm(pr2[7], pr2[6], 0x07050301u) & msk)};
        }
    }
}

// First layer, int32 path: u - 64 * 2^s from the wave's LDS base plus
// e W1[:, p], requantised to a - 64.
template <int KB1, int NT>
__device__ __forceinline__ void layer1_int32(const L1Loads<KB1, NT> &ld, const int (&ev)[NT], const int32_t *base32,
                                             int s1, int g, v4i (&a1)[NT][KB1]) {
    // wb repeats wa on this path; consuming it here keeps its loads beside
    // the others instead of being sunk into the packed path
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int kb = 0; kb < KB1; ++kb) asm volatile("" ::"v"(ld.wb[nt][kb]));
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int e = ev[nt];
#pragma unroll
        for (int kb = 0; kb < KB1; ++kb) {
            const int4 *bp = reinterpret_cast<const int4 *>(base32 + kb * 64 + g * 16);
            int out[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int4 bv = bp[t];
                const int w = ld.wa[nt][kb][t];
                v4i u = {bv.x + e * (int)(int8_t)(w & 0xff), bv.y + e * (int)(int8_t)((w >> 8) & 0xff),
                         bv.z + e * (int)(int8_t)((w >> 16) & 0xff), bv.w + e * (int)(int8_t)(w >> 24)};
                out[t] = requant4_offset(u, s1);
            }
            a1[nt][kb] = v4i{out[0], out[1], out[2], out[3]};
        }
    }
}

// The enumeration kernel.  L: weight layers (2 or 3); KB1 / KB2: 64-wide
// K-blocks of the first / second hidden layer; NT: 16-point N-tiles per
// chunk; WLDS: weight tiles of layers >= 2 staged in LDS (else read from
// global memory through the L2); EPI (3-layer nets): 1 for the fast hidden
// epilogue (shift[1] in {7, 8}), 0 for the general one; OUT16: at most 16
// classes (the output layer is one M-tile whose weights stay in registers,
// the second hidden layer streams into it, and decisions are taken from
// ballots against the clean label's logit; else the output layer loops over
// its M-tiles and every point takes the full argmax).
//
// Activations travel between layers in the offset form a - 64 (int8 in
// [-64, 63]; the fast epilogue's second hidden layer: a - 128); the offsets
// are folded into the next layer's bias.
template <int L, int KB1, int KB2, int NT, bool WLDS, int EPI, bool OUT16>
__global__ void __launch_bounds__(256, 2) enum_q8_kernel(EnumParams P, const int32_t *u0_store,
                                                      int64_t u0_stride, const int32_t *u0_index) {
    constexpr int CH = 16 * NT;
    constexpr int H1 = KB1 * 64;
    constexpr int H2 = KB2 * 64;
    constexpr int MT2 = (L == 3) ? H2 / 16 : 0;
    constexpr int KBL = (L == 3) ? KB2 : KB1;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const QNetDev &net = P.net;
    const int MTL = net.H[L] / 16;
    const int64_t w2_bytes = (L == 3) ? (int64_t)MT2 * KB1 * 1024 : 0;
    const int64_t wl_bytes = (int64_t)MTL * KBL * 1024;
    const int8_t *w2s = net.Wt[2];
    const int8_t *wls = net.Wt[L];
    // fast hidden epilogue (3-layer nets, shift[1] in {7, 8}): layer 1 emits
    // fast2 * (a1 - 64) (doubled bytes when fast2 == 2), layer 2 emits a2 - 128
    constexpr bool fast = (L == 3) && EPI == 1;
    const bool dbl1 = fast && net.fast2 == 2;
    // LDS: [weight tiles of layers >= 2 (WLDS)] [layer-2 init] [output init] [per-wave base]
    const int64_t wbytes = WLDS ? (w2_bytes + wl_bytes) : 0;
    const int nb2 = (L == 3) ? H2 : 0;
    const int nbl = net.H[L];
    {
        if constexpr (WLDS) {
            int4 *dst = reinterpret_cast<int4 *>(smem);
            const int64_t n2 = w2_bytes / 16, nl = wl_bytes / 16;
            for (int64_t t = threadIdx.x; t < n2; t += blockDim.x)
                dst[t] = reinterpret_cast<const int4 *>(net.Wt[2])[t];
            for (int64_t t = threadIdx.x; t < nl; t += blockDim.x)
                dst[n2 + t] = reinterpret_cast<const int4 *>(net.Wt[L])[t];
            w2s = reinterpret_cast<const int8_t *>(smem);
            wls = reinterpret_cast<const int8_t *>(smem) + w2_bytes;
        }
        int32_t *bdst = reinterpret_cast<int32_t *>(smem + wbytes);
        if constexpr (L == 3) {
            const int32_t *src2 = fast ? net.bf2 : net.bo[2];
            for (int t = threadIdx.x; t < nb2; t += blockDim.x) bdst[t] = src2[t];
        }
        const int32_t *srcl = fast ? net.bf3 : net.bo[L];
        for (int t = threadIdx.x; t < nbl; t += blockDim.x) bdst[nb2 + t] = srcl[t];
        __syncthreads();
    }
    const int32_t *b2s = reinterpret_cast<const int32_t *>(smem + wbytes);
    const int32_t *bls = b2s + nb2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j16 = lane & 15, g = lane >> 4;
    // per wave: one int32 base (int32 path) or kSegGroup int16 bases (packed path)
    constexpr int SLOT = (H1 * 4 > kSegGroup * H1 * 2) ? H1 * 4 : kSegGroup * H1 * 2;  // bytes
    char *wslot = smem + wbytes + 4 * (nb2 + nbl) + wave * SLOT;
    int32_t *base32 = reinterpret_cast<int32_t *>(wslot);
    int16_t *base16 = reinterpret_cast<int16_t *>(wslot);
    // per wave: the cursor record, after the four waves' slots
    Cursor *const cs = reinterpret_cast<Cursor *>(smem + wbytes + 4 * (nb2 + nbl) + 4 * SLOT) + wave_uniform(wave);

    // output layer of at most 16 classes: one M-tile, its weight tiles read
    // when needed, its init held in registers
    v4i bo4 = v4i{0, 0, 0, 0};
    if constexpr (OUT16) {
        const int4 b = *reinterpret_cast<const int4 *>(bls + g * 4);
        bo4 = v4i{b.x, b.y, b.z, b.w};
        // padding classes start (and, with zero weights, stay) at INT32_MIN
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (g * 4 + t >= net.dims[L]) bo4[t] = INT32_MIN;
    }

    const int s1 = net.shift[0];
    const int s2 = (L == 3) ? net.shift[1] : 0;
    const int ncls = net.dims[L];
    // general epilogue of layer 2: a2 - 64 = clamp(acc >> s2, -64, 63); the
    // bounds live in VGPRs so that the clamp is a single med3
    int lo2 = -64, hi2 = 63;
    asm("" : "+v"(lo2));
    asm("" : "+v"(hi2));
    // 32-bit pre-clamp of first-layer potentials for the packed base
    int ulo = 0, uhi = 0;
    if (P.packed) {
        const int f = net.f1;
        const int a0 = P.vb_lo + 16384, a1v = P.vb_hi + 16384;
        ulo = a0 >= 0 ? a0 / f : -((-a0 + f - 1) / f);   // floor(a0 / f)
        uhi = a1v >= 0 ? (a1v + f - 1) / f : -((-a1v) / f);  // ceil(a1v / f)
    }

    // ---- work distribution: first the leading single chunks, dealt out
    // statically round by round (wave g of the grid's NW waves takes chunks
    // g, g + NW, ...: the visiting order stays fine where an ordered search
    // meets its first counterexample, and no wave waits on the queue atomic,
    // which every wave of the grid hits at once when it starts), then
    // tickets from the global queue, each a batch of contiguous chunks (one
    // queue atomic, one cursor decode and one base per batch); the cursor
    // always describes the chunk whose first-layer loads are in flight.  Between chunks it rests in the wave's LDS record (read back
    // and written once per chunk), so that none of its fields holds
    // registers across the layers.
    int64_t cur_chunk = 0, end_chunk = 0;
    int fetches = 0;
    int sround = 0;  // static rounds taken
    const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t gwave = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave_uniform(wave);
    // next chunk of this wave; false when the queue is exhausted or a stop
    // or abort was requested.  seg: the segment (hence the base) changed.
    auto advance = [&](Cursor &c, bool first, bool &seg) __attribute__((always_inline)) -> bool {
        const EnumParams &Q = cold_params<EnumParams>();
        if (!first && ++cur_chunk < end_chunk) {
            seg = cursor_next<CH, EnumParams>(c, Q);
            return true;
        }
        // host-mapped abort request: polled on every 16th fetch of a wave,
        // never on its first (a grid whose waves all read host memory at once
        // waits on the bus), and before taking a ticket, so that every ticket
        // handed out is worked through (the queue counter then marks a
        // finished prefix of the chunks, the point a check resumes from)
        if (Q.abort_host && (++fetches & 15) == 0 && wave_uniform(*Q.abort_host)) return false;
        int64_t start = (int64_t)sround * n_waves + gwave, len = 1;
        if (start < Q.single) {
            ++sround;
        } else {
            unsigned long long ticket = 0;
            if (lane == 0) ticket = atomicAdd(Q.queue, 1ull);
            start = Q.resume + Q.single + (int64_t)wave_uniform(ticket) * Q.batch;  // lane 0's ticket
            len = Q.batch;
        }
        if (start >= Q.total_chunks) return false;
        if (wave_uniform(*Q.stop_flag)) {
            // an ordered search stops only past the earliest chunk known to
            // hold a counterexample, so every chunk before it is visited (a
            // stale read is too large: more work, never a skipped chunk)
            if (!Q.track_first) return false;
            const unsigned long long fc =
                wave_uniform(*reinterpret_cast<volatile unsigned long long *>(Q.first_chunk));
            if ((unsigned long long)start > fc) return false;
        }
        cur_chunk = start;
        end_chunk = min(start + len, Q.total_chunks);
        cursor_decode<CH, EnumParams>(c, Q, cur_chunk);
        seg = true;
        return true;
    };

    // state of the chunk at the cursor (prepared a chunk ahead)
    int label_n = -1, lowbits_n = 0, prop_n = -1;
    int valid_n[NT];  // 0 / 1 per lane, held in a VGPR (a lane mask would take two scalar registers)
    int plast_n[NT], ilast_n[NT];
    L1Loads<KB1, NT> ld;
    // segment set-up when needed (the group's bases in LDS slots, its
    // emission info in einfo_n), then positions and first-layer loads
    int nw_n = 1, einfo_n = 0;
    auto prepare = [&](const Cursor &c, bool seg) __attribute__((always_inline)) {
        const EnumParams &Q = cold_params<EnumParams>();
        if (seg) {
            const int32_t *u0s = u0_store + (int64_t)wave_uniform(u0_index[c.prop]) * u0_stride;
            Cursor ct = c;
            for (int w = 0; w < c.nw; ++w) {
                build_base<KB1>(ct, Q, u0s, base32, base16 + w * H1, lane, ulo, uhi);
                einfo_n = einfo_pack(make_emit_info<EnumParams>(ct, Q), w, einfo_n);
                if (w + 1 < c.nw) seg_step(ct);
            }
            nw_n = c.nw;
            __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): LDS writes done
            __builtin_amdgcn_wave_barrier();
        }
        if (c.prop != prop_n) {
            prop_n = c.prop;
            label_n = wave_uniform(Q.props[c.prop].label0);
            // bit t: this lane's class 4 g + t has a lower index than the label
            lowbits_n = 0;
#pragma unroll
            for (int t = 0; t < 4; ++t) lowbits_n |= (4 * g + t < label_n ? 1 : 0) << t;
        }
        einfo_n = lane_put(einfo_n, EI_GCLO, (int)(uint32_t)c.chunk);
        einfo_n = lane_put(einfo_n, EI_GCHI, (int)(c.chunk >> 32));
        const int obase = (int)c.ch * CH;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            valid_n[nt] = last_element32(c, Q, obase + nt * 16 + j16, plast_n[nt], ilast_n[nt]) ? 1 : 0;
            asm volatile("" : "+v"(valid_n[nt]));
        }
        layer1_issue<KB1, NT>(c, Q.net, Q.packed != 0, plast_n, ilast_n, g, ld);
    };

    // back to the LDS record: everything after a segment change, else the
    // chunk position; the clobber makes the next chunk read it back
    auto store_cursor = [&](const Cursor &c, bool full) __attribute__((always_inline)) {
        if (full) {
            *cs = c;
        } else {
            cs->chunk = c.chunk;
            cs->ch = c.ch;
        }
        asm volatile("" ::: "memory");
    };

    bool seg = false;
    {
        Cursor c;
        c.job = -1;
        if (!advance(c, true, seg)) return;
        prepare(c, seg);
        store_cursor(c, true);
    }
    RecOut ro;
    ro.next = 0;
    ro.end = 0;
    ro.slot = -1;
    ro.notified = false;
    ro.cex = 0;
    ro.ties = 0;

    while (true) {
        // ---- the current chunk is the prepared one: the same last-element
        // positions for each of the group's nw segments
        const int einfo = einfo_n;
        const int label0 = label_n, lowbits = lowbits_n;
        const int nw = nw_n;
        int valid[NT];
        int plast[NT], ilast[NT], ev[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            valid[nt] = valid_n[nt];
            plast[nt] = plast_n[nt];
            ilast[nt] = ilast_n[nt];
            ev[nt] = clamp_pixel(ld.xv[nt] + ld.dv[nt]) - ld.xv[nt];
        }
        bool more = true;
        for (int w = 0; w < nw; ++w) {

        // ---- layer 1: incremental update, requantisation, B operands
        v4i a1[NT][KB1];
        if (P.packed) {
            if (dbl1)  // uniform: one branch per segment
                layer1_packed<KB1, NT, true>(ld, ev, base16 + w * H1, g, a1);
            else
                layer1_packed<KB1, NT, false>(ld, ev, base16 + w * H1, g, a1);
        } else {
            layer1_int32<KB1, NT>(ld, ev, base32, s1, g, a1);
            if (dbl1) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                    for (int kb = 0; kb < KB1; ++kb)
#pragma unroll
                        for (int z = 0; z < 4; ++z) a1[nt][kb][z] = double_bytes(a1[nt][kb][z]);
            }
        }

        // ---- after the group's last segment has used them, the next chunk's
        // loads fly while this one goes through the MFMAs
        if (w == nw - 1) {
            Cursor c = *cs;
            more = advance(c, false, seg);
            if (more) {
                prepare(c, seg);
                store_cursor(c, seg);
            }
        }

        // ---- hidden layer 2 (L == 3): int8 MFMA, requantise into B operands;
        // with OUT16 every completed 64-row block of a2 goes straight into the
        // output layer's accumulators
        v4i acco[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acco[nt] = bo4;
        // weights read from global memory: the bases go through opaque
        // scalar copies here, inside the chunk loop; otherwise the compiler
        // hoists one 64-bit address per unrolled load (offsets beyond the
        // load's immediate field) out of the loop and spills them
        const int8_t *w2b = w2s, *wlb = wls;
        if constexpr (!WLDS) asm volatile("" : "+s"(w2b), "+s"(wlb));
        const v4i *wo = reinterpret_cast<const v4i *>(wlb) + lane;
        v4i a2[NT][(L == 3 && !OUT16) ? KB2 : 1];
        if constexpr (L == 3) {
            const v4i *wt2 = reinterpret_cast<const v4i *>(w2b) + lane;
            const int4 *bias2 = reinterpret_cast<const int4 *>(b2s + g * 4);
            v4i blk[NT];  // the a2 block being filled (OUT16)
            // requantisation of the finished tile pm into B operands; with
            // OUT16 every fourth tile completes a block for the output layer
            auto epilogue = [&](int pm, const v4i (&accf)[NT]) __attribute__((always_inline)) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    int q = fast ? requant4_sat(accf[nt]) : requant4_clamp(accf[nt], s2, lo2, hi2);
                    // pin the epilogue here: otherwise it is sunk towards the
                    // output layer, keeping every raw accumulator live
                    asm volatile("" : "+v"(q));
                    if constexpr (OUT16) blk[nt][pm & 3] = q;
                    else a2[nt][pm >> 2][pm & 3] = q;
                }
                if constexpr (OUT16) {
                    if ((pm & 3) == 3) {
                        const v4i w = wo[(pm >> 2) * 64];
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt)
                            acco[nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(w, blk[nt], acco[nt], 0, 0, 0);
                    }
                }
            };
            constexpr int EPI_V = (fast ? 5 : 11) * NT;  // VALU ops of one epilogue
            if constexpr (KB1 >= 2) {
                // Skewed software pipeline over the M-tiles.  Step mt runs the
                // first half of tile mt's K-blocks interleaved with the second
                // half of tile mt - 1's (2 NT independent accumulation chains,
                // enough to keep the matrix pipe busy), requantises tile mt - 2
                // (VALU between the MFMAs), and reads the next step's weight
                // tiles and init from LDS.
                constexpr int KH = KB1 / 2;
                v4i Alo[KH], Ahi[KH], Alo_n[KH], Ahi_n[KH];
#pragma unroll
                for (int kb = 0; kb < KH; ++kb) { Alo[kb] = wt2[kb * 64]; Ahi[kb] = Alo[kb]; }
                int4 bias = bias2[0], bnext = bias;
                v4i accA[NT], accE[NT];  // tile mt - 1 (finishing), tile mt - 2 (done)
#pragma unroll
                for (int mt = 0; mt <= MT2 + 1; ++mt) {
                    if (mt + 1 < MT2) {
#pragma unroll
                        for (int kb = 0; kb < KH; ++kb) Alo_n[kb] = wt2[((mt + 1) * KB1 + kb) * 64];
                        bnext = bias2[(mt + 1) * 4];
                    }
                    if (mt < MT2) {
#pragma unroll
                        for (int kb = 0; kb < KH; ++kb) Ahi_n[kb] = wt2[(mt * KB1 + KH + kb) * 64];
                    }
                    v4i accB[NT];
                    if (mt < MT2) {
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt) accB[nt] = v4i{bias.x, bias.y, bias.z, bias.w};
                    }
#pragma unroll
                    for (int kb = 0; kb < KH; ++kb) {
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt) {
                            if (mt >= 1 && mt <= MT2)
                                accA[nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(Ahi[kb], a1[nt][KH + kb], accA[nt], 0, 0, 0);
                            if (mt < MT2)
                                accB[nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(Alo[kb], a1[nt][kb], accB[nt], 0, 0, 0);
                        }
                    }
                    if (mt >= 2) {
                        epilogue(mt - 2, accE);
                        if (mt < MT2) {
                            // the next step's LDS reads first, then one MFMA and a
                            // share of the epilogue's VALU work, and so on
                            __builtin_amdgcn_sched_group_barrier(0x100, 2 * KH + 1, 0);
#pragma unroll
                            for (int i = 0; i < KB1 * NT; ++i) {
                                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                                __builtin_amdgcn_sched_group_barrier(0x002, (EPI_V + KB1 * NT - 1) / (KB1 * NT), 0);
                            }
                        }
                    }
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        accE[nt] = accA[nt];
                        accA[nt] = accB[nt];
                    }
#pragma unroll
                    for (int kb = 0; kb < KH; ++kb) {
                        Alo[kb] = Alo_n[kb];
                        Ahi[kb] = Ahi_n[kb];
                    }
                    bias = bnext;
                    __builtin_amdgcn_sched_barrier(0);
                }
            } else {
                // one K-block: the weight tile and init of tile mt + 1 are read
                // from LDS while tile mt computes, and the requantisation of
                // tile mt - 1 is interleaved with the MFMAs of tile mt
                v4i Acur = wt2[0], Anext = Acur;
                int4 bias = bias2[0], bnext = bias;
                v4i accp[NT];
#pragma unroll
                for (int mt = 0; mt <= MT2; ++mt) {
                    if (mt + 1 < MT2) {
                        Anext = wt2[(mt + 1) * 64];
                        bnext = bias2[(mt + 1) * 4];
                    }
                    v4i acc[NT];
                    if (mt < MT2) {
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt)
                            acc[nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(Acur, a1[nt][0],
                                                                           v4i{bias.x, bias.y, bias.z, bias.w}, 0, 0, 0);
                    }
                    if (mt > 0) {
                        epilogue(mt - 1, accp);
                        if (mt < MT2) {
                            __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
#pragma unroll
                            for (int i = 0; i < NT; ++i) {
                                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                                __builtin_amdgcn_sched_group_barrier(0x002, (EPI_V + NT - 1) / NT, 0);
                            }
                        }
                    }
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) accp[nt] = acc[nt];
                    Acur = Anext;
                    bias = bnext;
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        } else if constexpr (OUT16) {
#pragma unroll
            for (int kb = 0; kb < KBL; ++kb)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acco[nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(wo[kb * 64], a1[nt][kb], acco[nt], 0, 0, 0);
        }

        if constexpr (OUT16) {
            // ---- decisions from ballots against the clean label's logit zL:
            // a point is a counterexample iff some class c has z_c > zL, or
            // z_c == zL with c < label (padding classes sit at INT32_MIN); it is
            // an exact tie iff another class reaches zL.  Tiles with
            // counterexamples take the full argmax.
            // label-derived masks recomputed here with scalar ops (an opaque
            // copy of the label keeps the compiler from hoisting them out of
            // the loop, where they would only add to the scalar spills)
            int labv = label0;
            asm volatile("" : "+s"(labv));
            const int tL = labv & 3;
            const unsigned long long rowL = 0xffffull << (16 * (labv >> 2));
            bool mine[NT];
            int lab[NT];
            bool anyv = false;
            unsigned ties = 0;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const v4i z = acco[nt];
                const int zs = tL == 0 ? z[0] : tL == 1 ? z[1] : tL == 2 ? z[2] : z[3];
                const int zL = row_bcast(zs, labv >> 2);
                // common case first: no other class reaches zL (then the
                // point is neither a counterexample nor a tie)
                unsigned long long gem = 0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const unsigned long long ge = __ballot(z[t] >= zL);
                    gem |= (t == tL) ? (ge & ~rowL) : ge;
                }
                const unsigned vmask = (unsigned)(__ballot(valid[nt] != 0) & 0xffffull);
                unsigned viol16 = 0;
                mine[nt] = false;
                lab[nt] = 0;
                if (fold_groups(gem) & vmask) {
                    unsigned long long beat = 0, eqm = 0;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        // z_c beats zL iff z_c > zL - [c < label]
                        beat |= __ballot(z[t] > zL - ((lowbits >> t) & 1));
                        const unsigned long long eq = __ballot(z[t] == zL);
                        eqm |= (t == tL) ? (eq & ~rowL) : eq;
                    }
                    viol16 = fold_groups(beat) & vmask;
                    ties += __popc(fold_groups(eqm) & vmask & ~viol16);
                }
                if (viol16) {
                    anyv = true;
                    int bv = INT32_MIN, bi = 0x7fffffff, bc = 0;
                    argmax_tile<false>(z, 0, g, ncls, bv, bi, bc);
                    argmax_combine(bv, bi, bc);
                    mine[nt] = g == 0 && ((viol16 >> j16) & 1u);
                    lab[nt] = bi;
                    ties += (unsigned)__popcll(__ballot(mine[nt] && bc > 1));
                }
            }
            if (anyv) emit_tiles<NT>(ro, einfo, w, mine, plast, ilast, lab, lane);
            if (ties) rec_tally(ro, lane_get(einfo, EI_SLOT), 0u, ties, lane);
        } else {
            // ---- general output layer: M-tiles in turn, full lowest-index argmax
            int bestv[NT], besti[NT], bestc[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) { bestv[nt] = INT32_MIN; besti[nt] = 0x7fffffff; bestc[nt] = 0; }
            for (int mt = 0; mt < MTL; ++mt) {
                const int4 bias = *reinterpret_cast<const int4 *>(bls + mt * 16 + g * 4);
                v4i acc[NT];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[nt] = v4i{bias.x, bias.y, bias.z, bias.w};
#pragma unroll
                for (int kb = 0; kb < KBL; ++kb) {
                    const v4i A = *reinterpret_cast<const v4i *>(wlb + ((int64_t)(mt * KBL + kb) * 64 + lane) * 16);
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        if constexpr (L == 3)
                            acc[nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A, a2[nt][kb], acc[nt], 0, 0, 0);
                        else
                            acc[nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A, a1[nt][kb], acc[nt], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) argmax_tile<true>(acc[nt], mt, g, ncls, bestv[nt], besti[nt], bestc[nt]);
            }
            bool viol[NT];
            unsigned ties = 0;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                argmax_combine(bestv[nt], besti[nt], bestc[nt]);
                const bool mine = valid[nt] != 0 && g == 0;
                ties += (unsigned)__popcll(__ballot(mine && bestc[nt] > 1));
                viol[nt] = mine && besti[nt] != label0;
            }
            emit_tiles<NT>(ro, einfo, w, viol, plast, ilast, besti, lane);
            if (ties) rec_tally(ro, lane_get(einfo, EI_SLOT), 0u, ties, lane);
        }

        }  // segments of the group
        if (!more) break;
    }
    rec_finish(ro, lane);
}

#define IBMC_ENUM_VARIANT(L_, KB1_, KB2_, NT_, WLDS_, EPI_, O16_, TAG_)                                      \
    {L_, KB1_, KB2_, NT_, WLDS_, EPI_, O16_, 16 * NT_, "q8_L" #L_ "_kb" #KB1_ "x" #KB2_ "_nt" #NT_ "_" TAG_, \
     reinterpret_cast<const void *>(&enum_q8_kernel<L_, KB1_, KB2_, NT_, WLDS_, EPI_, O16_>)}
// instances for at most 16 classes
#define IBMC_VAR_LDS(L_, KB1_, KB2_, NT_) IBMC_ENUM_VARIANT(L_, KB1_, KB2_, NT_, true, 0, true, "lds")
#define IBMC_VAR_L2(L_, KB1_, KB2_, NT_) IBMC_ENUM_VARIANT(L_, KB1_, KB2_, NT_, false, 0, true, "l2")
#define IBMC_VAR_LDS_F(L_, KB1_, KB2_, NT_) IBMC_ENUM_VARIANT(L_, KB1_, KB2_, NT_, true, 1, true, "lds_f")
#define IBMC_VAR_L2_F(L_, KB1_, KB2_, NT_) IBMC_ENUM_VARIANT(L_, KB1_, KB2_, NT_, false, 1, true, "l2_f")
// instances for any number of classes
#define IBMC_VAR_LDS_G(L_, KB1_, KB2_, NT_, EPI_) IBMC_ENUM_VARIANT(L_, KB1_, KB2_, NT_, true, EPI_, false, "lds_g" #EPI_)
#define IBMC_VAR_L2_G(L_, KB1_, KB2_, NT_, EPI_) IBMC_ENUM_VARIANT(L_, KB1_, KB2_, NT_, false, EPI_, false, "l2_g" #EPI_)

}  // namespace ibmc
