// Work decomposition shared by the integer and the float enumeration
// kernels: a global chunk index maps to (job, segment, chunk in segment);
// a segment fixes every perturbed element but the last; the last element
// ranges over the segment's candidates, CH points per chunk.
#pragma once

#include "ibmc_internal.h"

namespace ibmc {

__device__ __forceinline__ int clamp_pixel(int v) { return min(max(v, 0), 255); }

// Load through a global-address-space pointer: pointers read from memory
// (the property's image and deltas, job tables) are generic to the compiler,
// and generic (flat) loads count against both memory and LDS waits.
template <class T>
__device__ __forceinline__ T gld(const T *p) {
    return *(const __attribute__((address_space(1))) T *)p;
}

// Values that are equal in every lane, made visibly uniform to the compiler
// (scalar registers and scalar branches instead of VGPRs and exec masks).
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ unsigned long long wave_uniform(unsigned long long v) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// The kernel's parameter block (its first argument) through a pointer that
// the compiler cannot see through: each call site re-reads the fields it
// needs with scalar loads, instead of the kernel holding them in registers
// from start to end.  For the rarely taken paths (queue, segment set-up,
// records).
template <class PT>
__device__ __forceinline__ const PT &cold_params() {
    typedef const __attribute__((address_space(4))) PT *cptr;
    cptr p = (cptr)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(p));
    return *(const PT *)p;
}

// Segment cursor: position of a wave in the global chunk order
// (job, last-prefix pixel q, prefix subset, prefix deltas, chunk).  All its
// fields are wave-uniform.
struct Cursor {
    int job, k, prop, slot, mode, m, n;
    int q;                 // last prefix pixel (plain k >= 2), -1 for k == 1
    int pre[kMaxK];        // prefix pixels pre[0..k-2] (pre[k-2] == q)
    int dg[kMaxK];         // prefix delta indices dg[0..k-2]
    int64_t shell;         // shell / list modes: shell index
    int64_t ch, nch;       // chunk inside the segment, chunks per segment
    int64_t seglen;        // candidates of the last element in this segment
    int64_t chunk;         // global chunk index
    int64_t job_end;
    const uint8_t *img;    // the property's image and delta set
    const int16_t *dl;
    unsigned mmagic;       // ceil(2^32 / m) for m >= 2, else 0 (see div_m)
    unsigned m1;           // m == 1
    int wseg;              // segments per group of this job
    int nw;                // segments in the current group (pre / dg: its first)
    int64_t s0, nseg;      // plain k >= 2: first segment of the group, segments of q
};


// lex_unrank_subset with a fixed trip count (kept in registers on the device).
__device__ __forceinline__ void lex_unrank_subset_fixed(int64_t rank, int k, int n, int (&p)[kMaxK]) {
    int64_t R = binom_small(n, k) - 1 - rank;
    int c = n;
#pragma unroll
    for (int j = 0; j < kMaxK; ++j) {
        if (j < k) {
            const int r = k - j;
            int cj = c - 1;
            while (cj >= r && binom_small(cj, r) > R) --cj;
            R -= binom_small(cj, r);
            p[j] = n - 1 - cj;
            c = cj;
        } else {
            p[j] = 0;
        }
    }
}

template <int CH, class PT>
__device__ __forceinline__ void cursor_job_start(Cursor &c, const PT &P, int job) {
    const EnumJob &J = P.jobs[job];
    c.job = job;
    c.k = wave_uniform(J.k);
    c.prop = wave_uniform(J.prop);
    c.slot = wave_uniform(J.slot);
    c.mode = wave_uniform(J.mode);
    c.m = wave_uniform(P.props[c.prop].m);
    c.n = wave_uniform(P.props[c.prop].n);
    c.job_end = (int64_t)wave_uniform((unsigned long long)J.chunk_end);
    c.img = reinterpret_cast<const uint8_t *>(wave_uniform((unsigned long long)P.props[c.prop].image));
    c.dl = P.props[c.prop].deltas;
    c.mmagic = c.m > 1 ? (unsigned)((0x100000000ull + (unsigned)c.m - 1) / (unsigned)c.m) : 0u;
    c.m1 = c.m == 1 ? 1u : 0u;
    c.wseg = max(1, wave_uniform(J.wseg));
    c.nw = 1;
    c.s0 = 0;
    c.nseg = 1;
}

template <int CH>
__device__ __forceinline__ void cursor_set_q(Cursor &c) {
    c.seglen = (int64_t)(c.n - 1 - c.q) * c.m;
    c.nch = (c.seglen + CH - 1) / CH;
}

// Decode global chunk `chunk` from scratch.
template <int CH, class PT>
__device__ __forceinline__ void cursor_decode(Cursor &c, const PT &P, int64_t chunk) {
    int lo = 0, hi = P.n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)wave_uniform((unsigned long long)P.jobs[mid].chunk_begin) <= chunk) lo = mid; else hi = mid - 1;
    }
    cursor_job_start<CH, PT>(c, P, lo);
    const EnumJob &J = P.jobs[lo];
    int64_t r = chunk - (int64_t)wave_uniform((unsigned long long)J.chunk_begin);
    c.chunk = chunk;
    if (c.mode == SEG_LIST1) {
        c.q = -1; c.shell = 0;
        c.seglen = (int64_t)c.n * c.m;
        c.nch = (c.seglen + CH - 1) / CH;
        c.ch = r;
        return;
    }
    if (c.mode == SEG_SHELL) {
        // shell_cum[t] = chunks before shell t; shells t >= 1 have t candidates
        int64_t N1 = (int64_t)c.n * c.m;
        int64_t a = 1, b = N1 - 1;
        while (a < b) {
            const int64_t mid = (a + b + 1) >> 1;
            if ((int64_t)wave_uniform((unsigned long long)J.shell_cum[mid]) <= r) a = mid; else b = mid - 1;
        }
        c.shell = a;
        c.seglen = a;
        c.nch = (a + CH - 1) / CH;
        c.ch = r - (int64_t)wave_uniform((unsigned long long)J.shell_cum[a]);
        return;
    }
    if (c.k == 1) {
        c.q = -1;
        c.seglen = (int64_t)c.n * c.m;
        c.nch = (c.seglen + CH - 1) / CH;
        c.ch = r;
        return;
    }
    // plain k >= 2: largest q in [k-2, n-2] with qcum[q] <= r
    int a = c.k - 2, b = c.n - 2;
    while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if ((int64_t)wave_uniform((unsigned long long)J.qcum[mid]) <= r) a = mid; else b = mid - 1;
    }
    c.q = a;
    cursor_set_q<CH>(c);
    const int64_t rr = r - (int64_t)wave_uniform((unsigned long long)J.qcum[a]);
    const int64_t grp = rr / c.nch;
    c.ch = rr % c.nch;
    int64_t mk1 = 1;
    for (int j = 0; j < c.k - 1; ++j) mk1 *= c.m;
    c.nseg = binom_small(a, c.k - 2) * mk1;
    c.s0 = grp * c.wseg;
    c.nw = (int)min<int64_t>(c.wseg, c.nseg - c.s0);
    const int64_t combo = c.s0 / mk1;
    int64_t dig = c.s0 % mk1;
#pragma unroll
    for (int j = kMaxK - 1; j >= 0; --j) {
        if (j < c.k - 1) { c.dg[j] = (int)(dig % c.m); dig /= c.m; }
    }
    int tmp[kMaxK];
    lex_unrank_subset_fixed(combo, c.k - 2, c.q, tmp);
#pragma unroll
    for (int j = 0; j < kMaxK; ++j) {
        if (j < c.k - 2) c.pre[j] = tmp[j];
        if (j == c.k - 2) c.pre[j] = c.q;
    }
}

// Step a plain (k >= 2) cursor to the next segment of the same q: prefix
// deltas with the last digit fastest, then the next (k-2)-subset of [0, q) in
// lexicographic order.  Returns false when q has no further segment (the
// deltas are then back at zero).
__device__ __forceinline__ bool seg_step(Cursor &c) {
    bool carry = true;
#pragma unroll
    for (int j = kMaxK - 1; j >= 0; --j) {
        if (carry && j < c.k - 1) {
            if (++c.dg[j] < c.m) carry = false;
            else c.dg[j] = 0;
        }
    }
    if (!carry) return true;
    const int r = c.k - 2;
    int piv = -1;
#pragma unroll
    for (int j = kMaxK - 1; j >= 0; --j)
        if (piv < 0 && j < r && c.pre[j] < c.q - (r - j)) piv = j;
    if (piv < 0) return false;
    int run = 0;
#pragma unroll
    for (int t = 0; t < kMaxK; ++t) {
        if (t == piv) { c.pre[t]++; run = c.pre[t]; }
        else if (t > piv && t < r) { run++; c.pre[t] = run; }
    }
    return true;
}

// Move to the next chunk.  Returns true when the segment (hence the base)
// changed.
template <int CH, class PT>
__device__ __forceinline__ bool cursor_next(Cursor &c, const PT &P) {
    c.chunk++;
    if (++c.ch < c.nch) return false;
    c.ch = 0;
    if (c.chunk >= c.job_end) {
        if (c.job + 1 < P.n_jobs) cursor_decode<CH, PT>(c, P, c.chunk);
        return true;
    }
    if (c.mode == SEG_SHELL) {
        c.shell++;
        c.seglen = c.shell;
        c.nch = (c.seglen + CH - 1) / CH;
        return true;
    }
    if (c.mode == SEG_LIST1 || c.k == 1) return true;  // single segment: end of job handled above
    // next group: step over this group's segments
    bool within = true;
    for (int t = 0; t < c.nw; ++t) within = seg_step(c);
    if (within) {
        c.s0 += c.nw;
        c.nw = (int)min<int64_t>(c.wseg, c.nseg - c.s0);
        return true;
    }
    // next q: first (k-2)-subset of [0, q), zero prefix deltas (already wrapped)
    const int r = c.k - 2;
    c.q++;
#pragma unroll
    for (int t = 0; t < kMaxK; ++t) {
        if (t < r) c.pre[t] = t;
        if (t == r) c.pre[t] = c.q;
    }
    cursor_set_q<CH>(c);
    int64_t mk1 = 1;
    for (int j = 0; j < c.k - 1; ++j) mk1 *= c.m;
    c.nseg = binom_small(c.q, r) * mk1;
    c.s0 = 0;
    c.nw = (int)min<int64_t>(c.wseg, c.nseg);
    return true;
}

// Resolve the last element of candidate position o of the current segment.
// Returns false when o is not a valid point.
template <class PT>
__device__ __forceinline__ bool last_element(const Cursor &c, const PT &P, int64_t o,
                                             int &p, int &i, int &pfirst, int &ifirst) {
    const EnumJob &J = P.jobs[c.job];
    if (o >= c.seglen) return false;
    if (c.mode == SEG_PLAIN) {
        p = c.q + 1 + (int)(o / c.m);
        i = (int)(o % c.m);
        return true;
    }
    const int cand = gld(J.order + o);
    p = cand / c.m;
    i = cand % c.m;
    if (c.mode == SEG_SHELL) {
        const int head = gld(J.order + c.shell);
        pfirst = head / c.m;
        ifirst = head % c.m;
        return p != pfirst;
    }
    return true;
}

// Quotient floor(x / m) for the per-point hot path: a multiply-high by
// M = ceil(2^32 / m) (cursor field mmagic) is exact for x < 2^32 / m, which
// holds for every candidate index (below n * |D| <= 2^24 here).  For m == 1,
// whose M does not fit 32 bits, mmagic is 0 and m1 is 1.
__device__ __forceinline__ unsigned div_m(const Cursor &c, unsigned x) {
    return __umulhi(x, c.mmagic) + x * c.m1;
}

// 32-bit form of last_element for the per-point hot path (segment lengths
// are below 2^31: at most n * |D| candidates).  Positions past the segment
// end report false and resolve to its first candidate, so that every lane
// reads in bounds.
template <class PT>
__device__ __forceinline__ bool last_element32(const Cursor &c, const PT &P, int o, int &p, int &i) {
    const bool ok = o < (int)c.seglen;
    const unsigned uo = ok ? (unsigned)o : 0u;
    if (c.mode == SEG_PLAIN) {
        const unsigned qd = div_m(c, uo);
        p = c.q + 1 + (int)qd;
        i = (int)(uo - qd * (unsigned)c.m);
        return ok;
    }
    const EnumJob &J = P.jobs[c.job];
    const int cand = gld(J.order + uo);
    const unsigned qd = div_m(c, (unsigned)cand);
    p = (int)qd;
    i = cand - (int)qd * c.m;
    if (c.mode == SEG_SHELL) {
        const int head = wave_uniform(gld(J.order + c.shell));
        return ok && p != (int)div_m(c, (unsigned)head);
    }
    return ok;
}

// Point rank (see the header) of a point given by its prefix and last element.
template <class PT>
__device__ __forceinline__ int64_t point_rank(const Cursor &c, const PT &P, int p, int i) {
    int pix[kMaxK], dig[kMaxK];
    int kk = c.k;
    if (c.mode == SEG_PLAIN) {
#pragma unroll
        for (int j = 0; j < kMaxK; ++j) {
            if (j < kk - 1) { pix[j] = c.pre[j]; dig[j] = c.dg[j]; }
            else if (j == kk - 1) { pix[j] = p; dig[j] = i; }
            else { pix[j] = 0; dig[j] = 0; }
        }
    } else if (c.mode == SEG_SHELL) {
        const int head = wave_uniform(P.jobs[c.job].order[c.shell]);
        const int ph = head / c.m, ih = head % c.m;
        if (ph < p) { pix[0] = ph; dig[0] = ih; pix[1] = p; dig[1] = i; }
        else { pix[0] = p; dig[0] = i; pix[1] = ph; dig[1] = ih; }
    } else {
        pix[0] = p; dig[0] = i;
    }
    int64_t d = 0, mk = 1, s = 0;
#pragma unroll
    for (int j = 0; j < kMaxK; ++j)
        if (j < kk) {
            d = d * c.m + dig[j];
            mk *= c.m;
            s += binom_small(c.n - 1 - pix[j], kk - j);
        }
    return (binom_small(c.n, kk) - 1 - s) * mk + d;
}

}  // namespace ibmc
