// Streamed tiles: the explicit step (velocity Verlet with the bond-force
// gather, critical-stretch damage and boundary data; Algorithm 4 with the
// force of Algorithm 1) over LDS tiles whose staging runs asynchronously, for
// one simulation or a batch of independent ones in the same launch; also the
// NP law's step and the two passes of the linear peridynamic solid's step
// (Algorithm 2: the state {m, theta}, then the force with the halo's per-node
// coefficients staged beside the records).
//
// Same tiles as the register-staged tile kernel (T consecutive sfc nodes,
// halo H_t, 16-bit tile-local bond words), but every global -> LDS copy is a
// gfx950 LDS DMA (global_load_lds_dword / _dwordx4): the data goes from L2
// straight into LDS without passing through registers, and no registers are
// held for prefetching, so two workgroups share each CU and cover each
// other's copy latency.
//
// Node state lives in HBM as one record per node, {x y z ux uy uz} (2-d:
// {x y ux uy}); a record is 3 (2) 16-byte chunks, so a halo record is three
// (two) DMA lanes.  The node update writes u^{k+1} into the u part of the
// other record buffer (the positions are never rewritten).
//
// A batch is a list of instances (StreamInst); their tiles are numbered one
// after the other and the persistent grid walks that list, so instances of
// any size share the launch.  The step index within a chunk is a launch
// argument (each captured launch of a hipGraph keeps its own), and the
// per-instance state at the start of the chunk sits in device descriptors,
// so a chunk of steps can be captured once and replayed.
//
// Per workgroup tile k: wait for this wave's copies, barrier (tile k and the
// ids of tile k+1 are in LDS); sum the bonds, one lane group per node in the
// gather kernel's summation order (so results are bit-identical to it),
// keeping what the node update needs from LDS in registers; barrier; issue
// the copies of tile k+1 and of the halo ids of tile k+2; then let L lanes of
// each group reduce their sums and update their node (kick, drift, boundary
// data), one component per lane, while those copies are in flight.  The bond
// words are read from global memory in the bond loop (one read per bond and
// pass; a break is stored at once), so they take no LDS.
#include <climits>

#include "pd_kernels.hpp"

namespace {

using namespace pdk;

typedef __attribute__((address_space(3))) char lds_char;

__device__ __forceinline__ uint32_t lds_addr(const void *p) {
    return (uint32_t)(uintptr_t)(const lds_char *)p;
}

// LDS DMA: lane l of the wave copies the 16 (4) bytes at base + voff into
// LDS at m0 + 16 l (m0 + 4 l).  m0 must be the same in every lane.  The copy
// is counted by the wave's vmcnt; dma_wait() waits for all of this wave's.
// The instructions are written out because the compiler's own form of them
// makes every later LDS read of the wave wait for the copy.
__device__ __forceinline__ void dma16(const void *base, uint32_t voff, uint32_t m0) {
    asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_dwordx4 %1, %0"
                 :
                 : "s"(base), "v"(voff), "s"(m0)
                 : "memory", "m0");
}
__device__ __forceinline__ void dma4(const void *base, uint32_t voff, uint32_t m0) {
    asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_dword %1, %0"
                 :
                 : "s"(base), "v"(voff), "s"(m0)
                 : "memory", "m0");
}
__device__ __forceinline__ void dma_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }


// an instance descriptor, read through the constant address space: scalar
// loads, which complete on their own counter and never wait for the tile
// copies or the node updates' stores in flight
typedef const __attribute__((address_space(4))) StreamInst *cinst;
__device__ __forceinline__ StreamInst load_inst(const StreamInst *base, uint32_t i) {
    const cinst p = (cinst)(uintptr_t)(base + i);
    StreamInst d;
    d.row_ptr = p->row_ptr;
    d.halo_ptr = p->halo_ptr;
    d.halo = p->halo;
    d.self_off = p->self_off;
    d.bw = p->bw;
    d.rec[0] = p->rec[0];
    d.rec[1] = p->rec[1];
    d.v = p->v;
    d.bc = p->bc;
    d.bc_vel = p->bc_vel;
    d.b = p->b;
    d.n = p->n;
    d.tile_begin = p->tile_begin;
    d.cv = p->cv;
    d.s_c = p->s_c;
    d.rho = p->rho;
    d.dt = p->dt;
    d.beta = p->beta;
    d.damage = p->damage;
    d.cur0 = p->cur0;
    d.vhalf0 = p->vhalf0;
    d.cd = p->cd;
    d.ramp = p->ramp;
    d.step0 = p->step0;
    d.limit = p->limit;
    return d;
}


// barrier that orders LDS only (global traffic in flight stays in flight)
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// per-tile metadata (32-bit words): h0, hn, b0 (even), b1, self offset,
// instance, first node, node count
constexpr int META = 8;
enum { MT_H0, MT_HN, MT_B0, MT_B1, MT_SO, MT_INST, MT_T0, MT_TN };
constexpr uint16_t BW_DEAD = 0x8000;

inline __host__ __device__ uint32_t round4(uint32_t x) { return (x + 3u) & ~3u; }

// the forms that stage the tile's velocities in LDS for the node update; the
// solid's force pass reads them from global memory instead (its LDS goes to
// the halo's coefficients), its state pass has no update
__host__ __device__ constexpr bool v_staged(int form) {
    return form == SK_LINEAR || form == SK_NP;
}
// bytes of the solid's coefficients {a, d} per node: float32 in mixed
// precision, float64 otherwise
__host__ __device__ constexpr uint32_t coef_bytes(int prec) { return prec == PD_MIXED ? 8u : 16u; }

// LDS layout, in this order (every region a multiple of 16 bytes): the tile
// slot (records, row offsets, v, boundary kinds), two halo-id slots, tile
// metadata, and for the solid's force pass the halo's coefficients {a, d}.
struct StreamLayout {
    uint32_t H, T, TP, VS, TB, MM, RD, US, SB;
    __host__ __device__ StreamLayout(int dim, uint32_t hcap, uint32_t tile, uint32_t mmax,
                                     int form, int prec) {
        H = hcap;                      // multiple of 32
        T = tile;
        TP = round4(tile + 1);         // row offsets
        TB = round4(tile / 4 + 1);     // 32-bit words of boundary kinds
        MM = round4(mmax * META);
        RD = dim == 3 ? 6 : 4;         // doubles per record
        US = dim == 3 ? 4 : 2;         // doubles per node in v
        VS = v_staged(form) ? tile * US : 0u;                        // doubles of v
        SB = form == SK_LPS_FORCE ? hcap * coef_bytes(prec) : 0u;    // bytes of {a, d}
    }
    __host__ __device__ size_t bytes() const {
        return (size_t)H * RD * 8 + (size_t)2 * H * 4 + (size_t)TP * 4 + (size_t)VS * 8 +
               (size_t)TB * 4 + (size_t)MM * 4 + (size_t)SB;
    }
};

__device__ __forceinline__ double ramp_of(double s, int64_t ramp) {
    if (ramp <= 0) return 1.0;
    const double r = s / (double)ramp;
    return r < 1.0 ? r : 1.0;
}

// BATCH = false: one simulation whose descriptor travels in the kernel
// arguments (sa.one); true: sa.ninst descriptors in device memory.  FORM:
// SK_LINEAR or SK_NP (one launch per step), SK_LPS_STATE (the solid's first
// pass: the coefficients {a, d} per node into I.lps, no update) or
// SK_LPS_FORCE (its force, with the neighbours' {a, d} staged beside the
// records, and the node update).
template <int DIM, int L, int PREC, bool BATCH, int FORM>
__global__ __launch_bounds__(1024) void stream_kernel(StreamArgs sa) {
    // PREC: PD_FP64, PD_MIXED, or PD_FP32 (float32 bond terms, compensated
    // float32 sums; linearised law only)
    constexpr bool MIXED = PREC == PD_MIXED, F32 = PREC == PD_FP32;
    static_assert(!F32 || FORM == SK_LINEAR, "PD_FP32: the linearised law only");
    extern __shared__ __attribute__((aligned(16))) double lds[];
    constexpr uint32_t RD = DIM == 3 ? 6 : 4, NCH = RD / 2, US = DIM == 3 ? 4 : 2;
    constexpr bool NP = FORM == SK_NP, LPS = FORM == SK_LPS_STATE || FORM == SK_LPS_FORCE;
    static_assert(!LPS || (DIM == 3 && !BATCH), "the solid: 3-d, single simulation");
    const StreamLayout lay(DIM, sa.hcap, sa.tile, sa.mmax, FORM, PREC);
    const uint32_t H = lay.H, T = lay.T;
    const uint32_t B = blockDim.x, tid = threadIdx.x, lane64 = tid & 63u;
    // first thread of this wave, in a scalar register: the copy loops below
    // then count and address in scalar registers
    const uint32_t wbase = __builtin_amdgcn_readfirstlane(tid - lane64);
    double *rec = lds;                                                           // H RD
    int32_t *ids = reinterpret_cast<int32_t *>(rec + (size_t)H * RD);            // 2 H
    uint32_t *rowp = reinterpret_cast<uint32_t *>(ids + (size_t)2 * H);          // TP
    double *vbuf = reinterpret_cast<double *>(rowp + lay.TP);                    // VS
    uint32_t *bcb = reinterpret_cast<uint32_t *>(vbuf + lay.VS);                 // TB
    uint32_t *meta = bcb + lay.TB;                                               // MM
    char *sps = reinterpret_cast<char *>(meta + lay.MM);                         // SB
    const StreamInst *inst = sa.inst;
    const int64_t s = sa.step;                          // step of this launch in its chunk
    // the record buffer holding u at this step
    auto cur_of = [&](const StreamInst &I) { return (uint32_t)((I.cur0 + s) & 1); };

    // persistent schedule: the tiles of this XCD's contiguous range, strided
    // over the XCD's workgroups
    const uint32_t nb = gridDim.x, x = blockIdx.x % 8, l = blockIdx.x / 8;
    const uint32_t gx = nb / 8 + (x < nb % 8 ? 1u : 0u);
    const uint32_t tq = sa.ntiles / 8, tr = sa.ntiles % 8;
    const uint32_t tbeg = x * tq + (x < tr ? x : tr), tcnt = tq + (x < tr ? 1u : 0u);
    const uint32_t K = l < tcnt ? (tcnt - l + gx - 1) / gx : 0u;
    if (K == 0) return;

    // metadata of every tile of this workgroup; tiles of instances that take
    // no step at this batch step get hn = 0 and are skipped
    for (uint32_t k = tid; k < K; k += B) {
        const uint32_t g = tbeg + l + k * gx;
        uint32_t lo = 0, hi = BATCH ? sa.ninst : 1u;   // last instance with tile_begin <= g
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (inst[mid].tile_begin <= g) lo = mid;
            else hi = mid;
        }
        const StreamInst I = BATCH ? load_inst(inst, lo) : sa.one;
        const uint32_t t = g - I.tile_begin, t0 = t * T, tn = min(T, I.n - t0);
        const uint32_t h0 = I.halo_ptr[t];
        uint32_t *m = meta + (size_t)k * META;
        m[MT_H0] = h0;
        m[MT_HN] = s < I.limit ? I.halo_ptr[t + 1] - h0 : 0u;
        m[MT_B0] = I.row_ptr[t0] & ~7u;   // 16-byte aligned bond-word copies
        m[MT_B1] = I.row_ptr[t0 + tn];   // (end of the tile's words)
        m[MT_SO] = I.self_off[t];
        m[MT_INST] = lo;
        m[MT_T0] = t0;
        m[MT_TN] = tn;
    }
    // descriptor of tile k's instance (the index is the same in every lane)
    auto inst_of = [&](uint32_t k) {
        if (!BATCH) return sa.one;
        return load_inst(inst, (uint32_t)__builtin_amdgcn_readfirstlane(meta[k * META + MT_INST]));
    };
    __syncthreads();

    // 3-d record copies: record (within a 64-record group) and byte offset
    // of chunk 64 p + lane of the group
    uint32_t crec[NCH], cpart[NCH];
#pragma unroll
    for (uint32_t p = 0; p < NCH; ++p) {
        const uint32_t x = 64u * p + lane64;
        crec[p] = x / NCH;
        cpart[p] = (x - crec[p] * NCH) * 16u;
    }
    // halo ids of tile k -> ids slot k mod 2
    auto issue_ids = [&](uint32_t k) {
        const StreamInst I = inst_of(k);
        const void *halo = I.halo;
        const uint32_t h0 = meta[k * META + MT_H0], hn = meta[k * META + MT_HN];
        int32_t *dst = ids + (size_t)(k & 1u) * H;
        for (uint32_t c0 = wbase; c0 < hn; c0 += B) {
            const uint32_t m0 = __builtin_amdgcn_readfirstlane(lds_addr(dst + c0));
            if (c0 + lane64 < hn) dma4(halo, (h0 + c0 + lane64) * 4u, m0);
        }
    };
    // records, row offsets, v and boundary kinds of tile k (the ids of tile k
    // are in ids slot k mod 2)
    auto issue_tile = [&](uint32_t k) {
        const uint32_t hn = meta[k * META + MT_HN];
        if (hn == 0) return;
        const uint32_t t0 = meta[k * META + MT_T0], tn = meta[k * META + MT_TN];
        const int32_t *hid = ids + (size_t)(k & 1u) * H;
        const StreamInst I = inst_of(k);
        const void *src = cur_of(I) ? I.rec[1] : I.rec[0];
        const void *rp = I.row_ptr, *vv = I.v, *bc = I.bc;
        if constexpr (NCH == 3) {
            // a wave copies 64 records per round in three copies of 64 lanes:
            // lane l of copy p moves 16-byte chunk 64 p + l of the group, whose
            // record and part are fixed per lane (no division per copy)
            for (uint32_t g0 = wbase; g0 < hn; g0 += B) {
#pragma unroll
                for (uint32_t p = 0; p < NCH; ++p) {
                    if (g0 + 64u * p / NCH >= hn) break;   // no record left for this copy
                    const uint32_t m0 = __builtin_amdgcn_readfirstlane(
                        lds_addr(rec + 2 * ((size_t)g0 * NCH + 64u * p)));
                    const uint32_t r = g0 + crec[p];
                    if (r < hn) dma16(src, (uint32_t)hid[r] * (RD * 8u) + cpart[p], m0);
                }
            }
        } else {
            const uint32_t nrc = hn * NCH;   // two chunks per record: a shift
            for (uint32_t c0 = wbase; c0 < nrc; c0 += B) {
                const uint32_t m0 = __builtin_amdgcn_readfirstlane(lds_addr(rec + 2 * (size_t)c0));
                const uint32_t c = c0 + lane64;
                if (c < nrc) {
                    const uint32_t r = c / NCH, part = c - r * NCH;
                    dma16(src, (uint32_t)hid[r] * (RD * 8u) + part * 16u, m0);
                }
            }
        }
        for (uint32_t c0 = wbase; c0 <= tn; c0 += B) {
            const uint32_t m0 = __builtin_amdgcn_readfirstlane(lds_addr(rowp + c0));
            if (c0 + lane64 <= tn) dma4(rp, (t0 + c0 + lane64) * 4u, m0);
        }
        // v (where staged) and the boundary kinds feed the node update (not in
        // the state pass)
        const uint32_t nvc = v_staged(FORM) ? tn * US / 2 : 0u;
        for (uint32_t c0 = wbase; c0 < nvc; c0 += B) {
            const uint32_t m0 = __builtin_amdgcn_readfirstlane(lds_addr(vbuf + 2 * (size_t)c0));
            if (c0 + lane64 < nvc) dma16(vv, (t0 * US + 2 * (c0 + lane64)) * 8u, m0);
        }
        const uint32_t nbw = FORM == SK_LPS_STATE ? 0u : (tn + 3) / 4;   // padded to words
        for (uint32_t c0 = wbase; c0 < nbw; c0 += B) {
            const uint32_t m0 = __builtin_amdgcn_readfirstlane(lds_addr(bcb + c0));
            if (c0 + lane64 < nbw) dma4(bc, t0 + 4 * (c0 + lane64), m0);
        }
        if constexpr (FORM == SK_LPS_FORCE) {
            // {a, d} of every halo node: one 16-byte copy each, or in mixed
            // precision two 4-byte copies (the float32 pair)
            const void *ls = I.lps;
            if constexpr (MIXED) {
                const uint32_t nsc = 2 * hn;
                for (uint32_t c0 = wbase; c0 < nsc; c0 += B) {
                    const uint32_t m0 = __builtin_amdgcn_readfirstlane(lds_addr(sps + 4 * (size_t)c0));
                    const uint32_t c = c0 + lane64;
                    if (c < nsc) dma4(ls, (uint32_t)hid[c >> 1] * 8u + (c & 1u) * 4u, m0);
                }
            } else {
                for (uint32_t c0 = wbase; c0 < hn; c0 += B) {
                    const uint32_t m0 = __builtin_amdgcn_readfirstlane(lds_addr(sps + 16 * (size_t)c0));
                    const uint32_t c = c0 + lane64;
                    if (c < hn) dma16(ls, (uint32_t)hid[c] * 16u, m0);
                }
            }
        }
    };

    // A tile's work in two phases around the barrier that frees its record
    // slot.  sums(k): the bond loops of tile k, the only phase that reads the
    // staged records, v and boundary kinds; what the node update needs from
    // LDS stays in registers.  update(k): the L lanes of each node's group
    // reduce their sums and update the node (kick, drift, boundary data, or
    // the central-difference update), one component per lane, with the same
    // arithmetic as node_update, while the copies of tile k + 1 are already in
    // flight.  The block holds T groups of L lanes: one node per group.  A
    // bond that breaks gets its dead bit in the global bond word at once.
    const uint32_t g = tid / L;
    const int lane = tid & (L - 1);
    std::conditional_t<F32, AccC, Acc64> acc;
    double ud_c = 0.0, vd_c = 0.0;   // this lane's component of u_i and v_i
    int kind_c = 0;
    auto sums = [&](uint32_t k) {
        acc = decltype(acc){};
        const uint32_t tn = meta[k * META + MT_TN], q = g;
        if (meta[k * META + MT_HN] == 0 || q >= tn) return;
        const StreamInst I = inst_of(k);
        const uint32_t t0 = meta[k * META + MT_T0];
        const uint32_t b0 = meta[k * META + MT_B0], so = meta[k * META + MT_SO];
        const double cv = I.cv, s_c = I.s_c, beta = I.beta;
        const float cv32 = (float)cv, s_c32 = (float)s_c;
        const int damage = I.damage;
        {
            const double *ri = rec + (size_t)(so + q) * RD;
            const double xix = ri[0], xiy = ri[1], xiz = DIM == 3 ? ri[2] : 0.0;
            const double uix = ri[DIM], uiy = ri[DIM + 1], uiz = DIM == 3 ? ri[DIM + 2] : 0.0;
            // the solid's force pass reads v from global memory, issued here so
            // that its latency overlaps the bond loop's first word loads
            double vg = 0.0;
            if constexpr (FORM == SK_LPS_FORCE)
                if (lane < (int)DIM) vg = I.v[(size_t)(t0 + q) * US + lane];
            const uint32_t rs = rowp[q] - b0, re = rowp[q + 1] - b0;
            // xi and eta of the bond whose word is w
            auto bond_vectors = [&](uint32_t w, double &dxx, double &dxy, double &dxz,
                                    double &dux, double &duy, double &duz) {
                const double2 *rj = reinterpret_cast<const double2 *>(
                    rec + (size_t)__builtin_amdgcn_ubfe(w, 0, 15) * RD);
                const double2 c0 = rj[0], c1 = rj[1];
                if (DIM == 3) {
                    const double2 c2 = rj[2];
                    dxx = c0.x - xix; dxy = c0.y - xiy; dxz = c1.x - xiz;
                    dux = c1.y - uix; duy = c2.x - uiy; duz = c2.y - uiz;
                } else {
                    dxx = c0.x - xix; dxy = c0.y - xiy; dxz = 0.0;
                    dux = c1.x - uix; duy = c1.y - uiy; duz = 0.0;
                }
            };
            // the words of this row come from global memory, two bonds per
            // pass (p and p + L, summed in that order: the gather kernel's
            // order), loaded two passes ahead into the register pair that pass
            // will use.  Reads past a row's end stay inside the padded array
            // and give valid record indices (the next rows' words, the next
            // tile's, or the dead pad); such a bond is masked off.
            const uint16_t *gw = I.bw + b0;
            const uint16_t *we = gw + re;
            const uint16_t *wq = gw + rs + lane;
            auto run_pairs = [&](auto &&pair) {
                auto pass = [&](uint32_t &ra, uint32_t &rb) {
                    const bool hb = wq + L < we;
                    const uint32_t wa = ra, wb = rb;
                    ra = wq[4 * L];
                    rb = wq[5 * L];
                    pair(wa, wb, hb);
                    wq += 2 * L;
                };
                uint32_t a0 = wq[0], b0w = wq[L], a1 = wq[2 * L], b1w = wq[3 * L];
                while (wq < we) {
                    pass(a0, b0w);
                    if (!(wq < we)) break;
                    pass(a1, b1w);
                }
            };
            if constexpr (FORM == SK_LPS_STATE) {
                // the solid's first pass, as lps_state_k: theta_i over live
                // bonds (uniform V_j), in the same order; m_i is fixed while
                // the bonds are (the solid takes no damage) and comes from the
                // gather kernel's state pass, run when the bonds were set
                const double m = lane == 0 ? I.lpsm[2 * (size_t)(t0 + q)] : 0.0;
                double sm = 0.0;
                run_pairs([&](uint32_t wa, uint32_t wb, bool hb) {
                    double ax, ay, az, aux, auy, auz, ar2, aq, aw;
                    double bx, by, bz, bux, buy, buz, br2, bq, bw;
                    bond_vectors(wa, ax, ay, az, aux, auy, auz);
                    bond_vectors(wb, bx, by, bz, bux, buy, buz);
                    if (!(wa & BW_DEAD)) {
                        asm volatile("" ::: "memory");
                        lps_terms<MIXED>(ax, ay, az, aux, auy, auz, ar2, aq, aw);
                        sm += aw;
                    }
                    if (hb && !(wb & BW_DEAD)) {
                        asm volatile("" ::: "memory");
                        lps_terms<MIXED>(bx, by, bz, bux, buy, buz, br2, bq, bw);
                        sm += bw;
                    }
                });
                // the uniform volume V is left out of the bond terms and
                // applied to each node's sums once
                sm = lane_sum<L>(sm) * I.vol;
                if (lane == 0) {
                    const LpsCoef qc =
                        lps_coef<MIXED>(m, m > 0.0 ? 3.0 / m * sm : 0.0, I.bulk, I.shear);
                    if constexpr (MIXED)
                        reinterpret_cast<float2 *>(I.lps)[t0 + q] =
                            make_float2((float)qc.a, (float)qc.d);
                    else
                        reinterpret_cast<double2 *>(I.lps)[t0 + q] = make_double2(qc.a, qc.d);
                }
                return;
            } else if constexpr (FORM == SK_LPS_FORCE) {
                // the solid's force, as the gather kernel's branch: the
                // scatter read from node i with {a, d} of both ends (a
                // dead bond adds nothing there either: its weight is 0)
                auto coef_of = [&](uint32_t j) {
                    LpsCoef r;
                    if constexpr (MIXED) {
                        const float2 ad = *reinterpret_cast<const float2 *>(sps + 8 * (size_t)j);
                        r.a = ad.x;
                        r.d = ad.y;
                    } else {
                        const double2 ad = *reinterpret_cast<const double2 *>(sps + 16 * (size_t)j);
                        r.a = ad.x;
                        r.d = ad.y;
                    }
                    return r;
                };
                const LpsCoef qi = coef_of(so + q);
                run_pairs([&](uint32_t wa, uint32_t wb, bool hb) {
                    double ax, ay, az, aux, auy, auz, ar2, aq, aw;
                    double bx, by, bz, bux, buy, buz, br2, bq, bw;
                    bond_vectors(wa, ax, ay, az, aux, auy, auz);
                    bond_vectors(wb, bx, by, bz, bux, buy, buz);
                    lps_terms<MIXED>(ax, ay, az, aux, auy, auz, ar2, aq, aw);
                    lps_terms<MIXED>(bx, by, bz, bux, buy, buz, br2, bq, bw);
                    const LpsCoef qa = coef_of(wa & 0x7fffu), qb = coef_of(wb & 0x7fffu);
                    if (!(wa & BW_DEAD)) {
                        asm volatile("" ::: "memory");
                        const double g = lps_force_weight(qi, qa, ar2, aq, aw, 1.0, true);
                        acc.x = fma(g, ax + aux, acc.x);
                        acc.y = fma(g, ay + auy, acc.y);
                        acc.z = fma(g, az + auz, acc.z);
                    }
                    if (hb && !(wb & BW_DEAD)) {
                        asm volatile("" ::: "memory");
                        const double g = lps_force_weight(qi, qb, br2, bq, bw, 1.0, true);
                        acc.x = fma(g, bx + bux, acc.x);
                        acc.y = fma(g, by + buy, acc.y);
                        acc.z = fma(g, bz + buz, acc.z);
                    }
                });
            } else {
                // a break is stored at once
                run_pairs([&](uint32_t wa, uint32_t wb, bool hb) {
                    double ax, ay, az, aux, auy, auz, bx, by, bz, bux, buy, buz;
                    bond_vectors(wa, ax, ay, az, aux, auy, auz);
                    bond_vectors(wb, bx, by, bz, bux, buy, buz);
                    bool ka, kb;
                    if constexpr (F32) {
                        float tax, tay, taz, tae, tbx, tby, tbz, tbe;
                        ka = bond32<DIM, false>(damage, s_c32, ax, ay, az, aux, auy, auz, cv32,
                                                (wa & BW_DEAD) != 0, tax, tay, taz, tae);
                        kb = bond32<DIM, false>(damage, s_c32, bx, by, bz, bux, buy, buz, cv32,
                                                !hb || (wb & BW_DEAD) != 0, tbx, tby, tbz, tbe);
                        pair_into<DIM, false>(acc, tax, tay, taz, tae, tbx, tby, tbz, tbe);
                    } else {
                        ka = bond<DIM, MIXED, false, NP>(damage, s_c, ax, ay, az, aux, auy, auz,
                                                         cv, (wa & BW_DEAD) != 0, acc, beta);
                        kb = bond<DIM, MIXED, false, NP>(damage, s_c, bx, by, bz, bux, buy, buz,
                                                         cv, !hb || (wb & BW_DEAD) != 0, acc,
                                                         beta);
                    }
                    // wq still addresses this pass's first bond
                    if (ka) *const_cast<uint16_t *>(wq) = (uint16_t)(wa | BW_DEAD);
                    if (kb) *const_cast<uint16_t *>(wq + L) = (uint16_t)(wb | BW_DEAD);
                });
            }
            if (lane < (int)DIM) {
                ud_c = lane == 0 ? uix : (lane == 1 ? uiy : uiz);
                vd_c = v_staged(FORM) ? vbuf[(size_t)q * US + lane] : vg;
                kind_c = (int)reinterpret_cast<const uint8_t *>(bcb)[q];
            }
        }
    };
    auto update = [&](uint32_t k) {
        const uint32_t tn = meta[k * META + MT_TN], q = g;
        if (FORM == SK_LPS_STATE || meta[k * META + MT_HN] == 0 || q >= tn) return;
        const StreamInst I = inst_of(k);
        const uint32_t t0 = meta[k * META + MT_T0];
        double *out = cur_of(I) ? I.rec[0] : I.rec[1];
        const int mode = (s > 0 || I.vhalf0) ? M_STEP_CONT : M_STEP_FIRST;
        const double r_half = ramp_of((double)(I.step0 + s) + 0.5, I.ramp);
        const double dt = I.dt, rho = I.rho;
        {
            double fx, fy, fz, Ue;
            if constexpr (F32) group_reduce_c<DIM, L, false>(acc, fx, fy, fz, Ue);
            else group_reduce<DIM, L, false>(acc, fx, fy, fz, Ue);
            if constexpr (FORM == SK_LPS_FORCE) {
                // the solid's weights left the uniform volume out
                fx = fx * I.vol;
                fy = fy * I.vol;
                fz = fz * I.vol;
            }
            if (lane < (int)DIM) {
                const uint32_t d = (uint32_t)lane, i = t0 + q;
                const double fd = d == 0 ? fx : (d == 1 ? fy : fz);
                const double ud = ud_c;
                double vd = vd_c;
                const int kind = kind_c;
                const double hdt = 0.5 * dt;
                double nd;
                if (kind == PD_BC_FREE && I.cd && s > 0) {
                    // central difference: the other record buffer still holds
                    // u^{k-1} (this lane's component is overwritten below)
                    const double bd = I.b ? I.b[(size_t)i * US + d] : 0.0;
                    const double pd = out[(size_t)i * RD + DIM + d];
                    nd = (2.0 * ud - pd) + dt * dt * (fd + bd) / rho;
                    vd = (nd - ud) / dt;
                } else if (kind == PD_BC_FREE) {
                    // the body-force load is used in its own branch, so no wait
                    // for it (nor for other loads in flight) lands on the path
                    // without one; fd + 0.0 == fd since the sums never end in -0.0
                    double fb = fd;
                    if (I.b) fb = fd + I.b[(size_t)i * US + d];
                    if (mode == M_STEP_CONT) vd = vd + hdt * fb / rho;
                    vd = vd + hdt * fb / rho;
                    nd = ud + dt * vd;
                } else if (kind == PD_BC_CLAMPED) {
                    vd = 0.0;
                    nd = 0.0;
                } else {
                    vd = r_half * I.bc_vel[(size_t)i * US + d];
                    nd = ud + dt * vd;
                }
                I.v[(size_t)i * US + d] = vd;
                out[(size_t)i * RD + DIM + d] = nd;
            }
        }
    };

    issue_ids(0);
    if (K > 1) issue_ids(1);
    dma_wait();
    __syncthreads();
    issue_tile(0);
    for (uint32_t k = 0; k < K; ++k) {
        dma_wait();
        lds_barrier();                       // tile k and the ids of tile k+1 are in LDS
        sums(k);
        lds_barrier();                       // the slot is free once the sums are done
        if (k + 1 < K) issue_tile(k + 1);
        if (k + 2 < K) issue_ids(k + 2);
        update(k);
    }
}

template <int DIM, int L, int FORM>
void *pick_lp(int prec, bool batch) {
    if (batch) {
        if constexpr (FORM == SK_LINEAR) {
            if (prec == PD_FP32) return (void *)stream_kernel<DIM, L, PD_FP32, true, FORM>;
        }
        if constexpr (FORM == SK_LINEAR || FORM == SK_NP)
            return prec == PD_MIXED ? (void *)stream_kernel<DIM, L, PD_MIXED, true, FORM>
                                    : (prec == PD_FP64
                                           ? (void *)stream_kernel<DIM, L, PD_FP64, true, FORM>
                                           : nullptr);
        return nullptr;
    }
    if constexpr (FORM == SK_LINEAR) {
        if (prec == PD_FP32) return (void *)stream_kernel<DIM, L, PD_FP32, false, FORM>;
    }
    return prec == PD_MIXED ? (void *)stream_kernel<DIM, L, PD_MIXED, false, FORM>
                            : (prec == PD_FP64 ? (void *)stream_kernel<DIM, L, PD_FP64, false, FORM>
                                               : nullptr);
}

// the kernel of a form: lanes 2..32, each precision, single or batch (the
// solid: 3-d, single simulation only; PD_FP32: the linearised law)
template <int DIM, int FORM>
void *pick_form(int lanes, int prec, bool batch) {
    switch (lanes) {
    case 2: return pick_lp<DIM, 2, FORM>(prec, batch);
    case 4: return pick_lp<DIM, 4, FORM>(prec, batch);
    case 8: return pick_lp<DIM, 8, FORM>(prec, batch);
    case 16: return pick_lp<DIM, 16, FORM>(prec, batch);
    case 32: return pick_lp<DIM, 32, FORM>(prec, batch);
    default: return nullptr;
    }
}

template <int DIM>
void *pick_stream(int lanes, int prec, bool batch, int form) {
    switch (form) {
    case SK_LINEAR: return pick_form<DIM, SK_LINEAR>(lanes, prec, batch);
    case SK_NP: return pick_form<DIM, SK_NP>(lanes, prec, batch);
    case SK_LPS_STATE:
        if constexpr (DIM == 3) return pick_form<3, SK_LPS_STATE>(lanes, prec, batch);
        return nullptr;
    case SK_LPS_FORCE:
        if constexpr (DIM == 3) return pick_form<3, SK_LPS_FORCE>(lanes, prec, batch);
        return nullptr;
    default: return nullptr;
    }
}

// records {x y z ux uy uz} (2-d {x y ux uy}) from xv and u
template <int DIM>
__global__ void rec_pack_k(uint32_t n, const double *xv, const double *u, double *rec) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int RD = DIM == 3 ? 6 : 4, US = DIM == 3 ? 4 : 2;
    for (int d = 0; d < DIM; ++d) {
        rec[(size_t)i * RD + d] = xv[4 * (size_t)i + d];
        rec[(size_t)i * RD + DIM + d] = u[(size_t)i * US + d];
    }
}

template <int DIM>
__global__ void rec_unpack_k(uint32_t n, const double *rec, double *u) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int RD = DIM == 3 ? 6 : 4, US = DIM == 3 ? 4 : 2;
    for (int d = 0; d < US; ++d) u[(size_t)i * US + d] = d < DIM ? rec[(size_t)i * RD + DIM + d] : 0.0;
}

}  // namespace

// Launch geometry of the streamed kernel for ntiles tiles in total; false if
// it cannot run this layout.
bool pd_stream_geometry(pd_ctx ctx, int dim, uint32_t ntiles, uint32_t tile, uint32_t hcap,
                        uint32_t bcap, int lanes, int prec, bool batch, int form, int *block,
                        unsigned *grid, uint32_t *mmax, size_t *lds) {
    const uint32_t B = tile * (uint32_t)lanes;
    if (B < 64 || B > 1024 || B % 64 != 0) return false;
    if (lanes < dim) return false;   // the node update takes one lane per component
    (void)bcap;                      // the bond words stay in global memory
    void *k = dim == 3 ? pick_stream<3>(lanes, prec, batch, form)
                       : pick_stream<2>(lanes, prec, batch, form);
    if (!k) return false;
    for (int pass = 0; pass < 2; ++pass) {
        // first pass: one workgroup per CU gives the tile bound; second pass:
        // as many per CU as LDS and registers allow
        unsigned g = (unsigned)ctx->num_cu;
        if (pass == 1) {
            int per_cu = 0;
            const size_t bytes = StreamLayout(dim, hcap, tile, *mmax, form, prec).bytes();
            (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k, (int)B,
                                                             bytes) != hipSuccess)
                return false;
            if (per_cu < 1) return false;
            g = (unsigned)(ctx->num_cu * per_cu);
        }
        if (g > ntiles) g = ntiles;
        if (g < 8 && ntiles >= 8) g = 8;
        if (g < 1) g = 1;
        uint32_t m = 0;
        for (uint32_t x = 0; x < 8; ++x) {
            const uint32_t gx = g / 8 + (x < g % 8 ? 1u : 0u);
            const uint32_t tc = ntiles / 8 + (x < ntiles % 8 ? 1u : 0u);
            if (gx == 0) {
                if (tc) return false;
                continue;
            }
            const uint32_t kk = (tc + gx - 1) / gx;
            if (kk > m) m = kk;
        }
        const size_t bytes = StreamLayout(dim, hcap, tile, m, form, prec).bytes();
        if (bytes > 160 * 1024) return false;
        *mmax = m;
        *lds = bytes;
        *grid = g;
    }
    *block = (int)B;
    return true;
}

// a neighbour list's record and copy offsets fit the kernel's 32-bit forms
bool pd_stream_fits(int dim, uint32_t n, uint64_t nnz, uint64_t halo_total) {
    const uint64_t RB = dim == 3 ? 48u : 32u;
    return (uint64_t)n * RB < (1ull << 32) && 2 * nnz + 16 < (1ull << 32) &&
           halo_total * 4 < (1ull << 32);
}

int pd_launch_stream(pd_ctx ctx, hipStream_t st, int dim, const StreamArgs &sa, int lanes,
                     int prec, int form, int block, unsigned grid, size_t lds) {
    const bool batch = sa.inst != nullptr;
    void *k = dim == 3 ? pick_stream<3>(lanes, prec, batch, form)
                       : pick_stream<2>(lanes, prec, batch, form);
    if (!k) return pd_set_error(ctx, PD_EINVAL, "no streamed kernel of form %d for %d lanes", form,
                                lanes);
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    StreamArgs args = sa;
    void *argv[] = {&args};
    PD_HIP(ctx, hipLaunchKernel(k, dim3(grid), dim3(block), argv, lds, st));
    return PD_OK;
}


int pd_rec_pack(pd_ctx ctx, int dim, uint32_t n, const double *xv, const double *u, double *rec) {
    if (dim == 3) rec_pack_k<3><<<pd_blocks(n), PD_BLOCK, 0, ctx->stream>>>(n, xv, u, rec);
    else rec_pack_k<2><<<pd_blocks(n), PD_BLOCK, 0, ctx->stream>>>(n, xv, u, rec);
    PD_LAUNCH_CHECK(ctx);
    return PD_OK;
}

int pd_rec_unpack(pd_ctx ctx, int dim, uint32_t n, const double *rec, double *u) {
    if (dim == 3) rec_unpack_k<3><<<pd_blocks(n), PD_BLOCK, 0, ctx->stream>>>(n, rec, u);
    else rec_unpack_k<2><<<pd_blocks(n), PD_BLOCK, 0, ctx->stream>>>(n, rec, u);
    PD_LAUNCH_CHECK(ctx);
    return PD_OK;
}
