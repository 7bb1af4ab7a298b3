// fragment.hip -- the linear-time meta-heuristic of Sec. I with fixed-sweep
// simulated annealing as the subsystem optimiser: the lattice is tiled by
// cores of c^3 spins, each core is decimated from anneals of the l^3
// fragment around it (l = c + 2h), and fragments overlap the cores decimated
// before them, which act as fixed boundary spins (the bootstrapping of
// App. C).  Cores are processed in phases; all cores of a phase run at once
// and see the decimation state at the start of their phase.
//
// One launch per phase, one work group per (core, run).  The group's R
// waves anneal R independent copies of the fragment in LDS (wave r = copy
// r), each on its own without block barriers: the spins of its copy, the
// fragment's in-fragment couplings and per-colour lists of the free sites
// with their neighbours stay on chip for the whole anneal.  The copy with the
// lowest in-fragment energy (lowest r among equals) gives the core's spins.
// A fragment site counts as fixed exactly when its core belongs to an
// earlier phase, so a group never reads the cores written in its own phase.
#include "common.hpp"
#include "variants.hpp"

namespace sg {

constexpr int kFragMaxL = SG_FRAG_MAX_L;
constexpr int kFragMaxR = SG_FRAG_MAX_R;
constexpr int kFragMaxSites = kFragMaxL * kFragMaxL * kFragMaxL;

struct FragJob {
    const int8_t *J;        // natural-order couplings [6][N]
    const uint32_t *thr;    // [S][K]
    int8_t *dec;            // [n_runs][N], 0 = not yet decimated
    int32_t L, c, h, l, nb, P, order, R, S, K;
    uint32_t run0, k0, k1;
};

__host__ __device__ inline int frag_phase(const FragJob &j, int bx, int by, int bz)
{
    return j.order == 0 ? (bx % j.P) + j.P * ((by % j.P) + j.P * (bz % j.P)) : bx + by + bz;
}

__host__ __device__ inline int frag_phases(const FragJob &j)
{
    return j.order == 0 ? j.P * j.P * j.P : 3 * (j.nb - 1) + 1;
}

__host__ __device__ inline int imax(int a, int b) { return a > b ? a : b; }
__host__ __device__ inline int imin(int a, int b) { return a < b ? a : b; }

// number of (by) with 0 <= by < nb and 0 <= q - bx - by < nb
__host__ __device__ inline int wave_row(int nb, int q, int bx)
{
    const int lo = imax(0, q - bx - (nb - 1)), hi = imin(nb - 1, q - bx);
    return hi >= lo ? hi - lo + 1 : 0;
}

__host__ __device__ inline int frag_phase_count(const FragJob &j, int q)
{
    if (j.order == 0) {
        const int m = j.nb / j.P;
        return m * m * m;
    }
    int n = 0;
    for (int bx = 0; bx < j.nb; ++bx) n += wave_row(j.nb, q, bx);
    return n;
}

// core (bx, by, bz) of the idx-th core of phase q
__device__ inline void frag_phase_core(const FragJob &j, int q, int idx, int &bx, int &by, int &bz)
{
    if (j.order == 0) {
        const int m = j.nb / j.P;
        bx = q % j.P + j.P * (idx % m);
        by = (q / j.P) % j.P + j.P * ((idx / m) % m);
        bz = q / (j.P * j.P) + j.P * (idx / (m * m));
        return;
    }
    for (bx = 0; bx < j.nb; ++bx) {
        const int n = wave_row(j.nb, q, bx);
        if (idx < n) break;
        idx -= n;
    }
    by = imax(0, q - bx - (j.nb - 1)) + idx;
    bz = q - bx - by;
}

// Orders one wave's LDS accesses across this point (a memory fence at
// wavefront scope for the compiler, then the wave barrier)
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// A free site of one colour, as the sweep reads it: its local index and its
// six neighbours' (the site itself where the neighbour is outside the
// fragment: its coupling is zero there)
struct FragSite {
    uint16_t j, nb[6];
    uint16_t pad;
};

__global__ __launch_bounds__(kFragMaxR * 64) void k_frag_phase(FragJob job, int q, int count)
{
    __shared__ int8_t s_spin[kFragMaxR][kFragMaxSites];
    __shared__ int8_t s_J[6][kFragMaxSites];
    __shared__ uint8_t s_free[kFragMaxSites];
    __shared__ FragSite s_site[kFragMaxSites];          // free sites, colour 0 then colour 1
    __shared__ uint32_t s_thr[kFragMaxR][SG_K_MAX];    // each wave's copy of the current row
    __shared__ int32_t s_E[kFragMaxR];
    __shared__ int32_t s_nsite[2];
    __shared__ int32_t s_best;

    const int tid = static_cast<int>(threadIdx.x);
    const int NT = static_cast<int>(blockDim.x);   // R * 64
    const int run_i = static_cast<int>(blockIdx.x) / count;
    const int idx = static_cast<int>(blockIdx.x) - run_i * count;
    const int L = job.L, c = job.c, h = job.h, l = job.l, nb = job.nb;
    const int n3 = l * l * l;
    const int64_t N = static_cast<int64_t>(L) * L * L;
    int bx, by, bz;
    frag_phase_core(job, q, idx, bx, by, bz);
    const uint32_t k = static_cast<uint32_t>(bx + nb * (by + nb * bz));
    const uint32_t run = job.run0 + static_cast<uint32_t>(run_i);
    int8_t *dec = job.dec + static_cast<int64_t>(run_i) * N;
    const int ox = bx * c - h, oy = by * c - h, oz = bz * c - h;
    // parity of the global coordinates of local site (0,0,0) (L is even, so
    // the periodic wrap keeps parities)
    const int opar = (ox + oy + oz) & 1;

    // ---- fragment set-up: free/fixed, in-fragment couplings, copies --------
    for (int j = tid; j < n3; j += NT) {
        const int lx = j % l, ly = (j / l) % l, lz = j / (l * l);
        const int gx = (ox + lx + L) % L, gy = (oy + ly + L) % L, gz = (oz + lz + L) % L;
        const int64_t g = gx + static_cast<int64_t>(L) * (gy + static_cast<int64_t>(L) * gz);
        const bool fixed = frag_phase(job, gx / c, gy / c, gz / c) < q;
        s_free[j] = fixed ? 0 : 1;
        const int8_t v = fixed ? dec[g] : 0;
        for (int r = 0; r < job.R; ++r) s_spin[r][j] = v;
        const bool in[6] = {lx + 1 < l, lx > 0, ly + 1 < l, ly > 0, lz + 1 < l, lz > 0};
#pragma unroll
        for (int d = 0; d < 6; ++d) s_J[d][j] = in[d] ? job.J[d * N + g] : 0;
    }
    __syncthreads();
    // lists of the free sites of each colour (wave 0, 64 sites per ballot)
    if (tid < 64) {
        int base = 0;
        for (int col = 0; col < 2; ++col) {
            for (int j0 = 0; j0 < n3; j0 += 64) {
                const int j = j0 + tid;
                bool take = false;
                int lx = 0, ly = 0, lz = 0;
                if (j < n3) {
                    lx = j % l;
                    ly = (j / l) % l;
                    lz = j / (l * l);
                    take = s_free[j] && ((opar + lx + ly + lz) & 1) == col;
                }
                const uint64_t mask = __ballot(take);
                if (take) {
                    const int pos = base + __popcll(mask & ((1ull << tid) - 1ull));
                    FragSite fs;
                    fs.j = static_cast<uint16_t>(j);
                    fs.nb[0] = static_cast<uint16_t>(lx + 1 < l ? j + 1 : j);
                    fs.nb[1] = static_cast<uint16_t>(lx > 0 ? j - 1 : j);
                    fs.nb[2] = static_cast<uint16_t>(ly + 1 < l ? j + l : j);
                    fs.nb[3] = static_cast<uint16_t>(ly > 0 ? j - l : j);
                    fs.nb[4] = static_cast<uint16_t>(lz + 1 < l ? j + l * l : j);
                    fs.nb[5] = static_cast<uint16_t>(lz > 0 ? j - l * l : j);
                    fs.pad = 0;
                    s_site[pos] = fs;
                }
                base += __popcll(mask);
            }
            if (tid == 0) s_nsite[col] = base;   // end of colour col's list
        }
    }
    for (int p = tid; p < job.R * n3; p += NT) {
        const int r = p / n3, j = p - r * n3;
        if (s_free[j]) {
            const Rand4 u = philox10(static_cast<uint32_t>(r * n3 + j), 0xFFFFFFFFu, k, run, job.k0, job.k1);
            s_spin[r][j] = (u.w[0] >> 31) ? -1 : 1;
        }
    }
    __syncthreads();

    // ---- sweeps: wave r anneals copy r on its own ------------------------------
    // Nothing below is shared between waves until the energies, so the waves
    // need no block barrier: a wave's LDS accesses execute in issue order,
    // and wave_sync keeps the compiler from moving them across a phase.
    const int r = tid >> 6, lane = tid & 63;
    int8_t *sp = s_spin[r];
    uint32_t *thr_r = s_thr[r];
    const int n0 = s_nsite[0], n01 = s_nsite[1];
    // the first row; each sweep fetches the next row while it runs
    if (lane < job.K && job.S > 0) thr_r[lane] = job.thr[lane];
    wave_sync();
    // The uniforms of site j in sweeps 4m..4m+3 are the four words of one
    // Philox call with counter (r l^3 + j, 2m + colour, core, run).
    auto draws = [&](int j, int s, int col) {
        return philox10(static_cast<uint32_t>(r * n3 + j), 2u * static_cast<uint32_t>(s >> 2) + static_cast<uint32_t>(col),
                        k, run, job.k0, job.k1);
    };
    auto word = [](const Rand4 &u, int i) { return i == 0 ? u.w[0] : i == 1 ? u.w[1] : i == 2 ? u.w[2] : u.w[3]; };
    // One Metropolis proposal: the site's record and couplings come from fs
    // and Jd (registers or LDS); u4 holds the site's draws of this block of
    // four sweeps, or is null to draw them here.
    auto propose = [&](const FragSite &fs, const int8_t *Jd, int s, int col, const Rand4 *u4) {
        const int j = fs.j;
        int hf = 0;
#pragma unroll
        for (int d = 0; d < 6; ++d) hf += Jd[d] * sp[fs.nb[d]];
        const int kk = -sp[j] * hf;
        bool acc = kk <= 0;
        // a zero threshold rejects every draw: no need to draw
        if (!acc && kk <= job.K && thr_r[kk - 1] != 0u)
            acc = word(u4 ? *u4 : draws(j, s, col), s & 3) < thr_r[kk - 1];
        if (acc) sp[j] = static_cast<int8_t>(-sp[j]);
    };
    if (n0 <= 64 && n01 - n0 <= 64) {
        // at most one site per lane and colour (l = 5 single-spin fragments):
        // each lane keeps its two sites' records and couplings in registers
        FragSite mine[2];
        int8_t mj[2][6];
        bool have[2];
#pragma unroll
        for (int col = 0; col < 2; ++col) {
            const int e = (col ? n0 : 0) + lane;
            have[col] = e < (col ? n01 : n0);
            mine[col] = have[col] ? s_site[e] : FragSite{};   // a zeroed record reads site 0
#pragma unroll
            for (int d = 0; d < 6; ++d) mj[col][d] = s_J[d][mine[col].j];
        }
        Rand4 u4[2] = {};
        for (int s = 0; s < job.S; ++s) {
            const uint32_t next = (lane < job.K && s + 1 < job.S)
                                      ? job.thr[static_cast<int64_t>(s + 1) * job.K + lane] : 0u;
            if ((s & 3) == 0) {
#pragma unroll
                for (int col = 0; col < 2; ++col)
                    if (have[col]) u4[col] = draws(mine[col].j, s, col);
            }
#pragma unroll
            for (int col = 0; col < 2; ++col) {
                if (have[col]) propose(mine[col], mj[col], s, col, &u4[col]);
                wave_sync();
            }
            if (lane < job.K && s + 1 < job.S) thr_r[lane] = next;
            wave_sync();
        }
    } else {
        for (int s = 0; s < job.S; ++s) {
            const uint32_t next = (lane < job.K && s + 1 < job.S)
                                      ? job.thr[static_cast<int64_t>(s + 1) * job.K + lane] : 0u;
            for (int col = 0; col < 2; ++col) {
                const int e0 = col ? n0 : 0, e1 = col ? n01 : n0;
                for (int e = e0 + lane; e < e1; e += 64) {
                    const FragSite fs = s_site[e];
                    int8_t Jd[6];
#pragma unroll
                    for (int d = 0; d < 6; ++d) Jd[d] = s_J[d][fs.j];
                    propose(fs, Jd, s, col, nullptr);
                }
                wave_sync();
            }
            if (lane < job.K && s + 1 < job.S) thr_r[lane] = next;
            wave_sync();
        }
    }

    // ---- the copy with the lowest in-fragment energy gives the core -----------
    int e = 0;
    for (int j = lane; j < n3; j += 64) {
        const int lx = j % l, ly = (j / l) % l, lz = j / (l * l);
        if (lx + 1 < l) e += s_J[0][j] * sp[j] * sp[j + 1];
        if (ly + 1 < l) e += s_J[2][j] * sp[j] * sp[j + l];
        if (lz + 1 < l) e += s_J[4][j] * sp[j] * sp[j + l * l];
    }
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
    if (lane == 0) s_E[r] = e;
    __syncthreads();
    if (tid == 0) {
        int best = 0;
        for (int i = 1; i < job.R; ++i)
            if (s_E[i] < s_E[best]) best = i;
        s_best = best;
    }
    __syncthreads();
    const int8_t *bs = s_spin[s_best];
    for (int p = tid; p < c * c * c; p += NT) {
        const int cx = p % c, cy = (p / c) % c, cz = p / (c * c);
        const int j = (h + cx) + l * ((h + cy) + l * (h + cz));
        const int64_t g = (bx * c + cx) + static_cast<int64_t>(L) * ((by * c + cy) + static_cast<int64_t>(L) * (bz * c + cz));
        dec[g] = bs[j];
    }
}

__global__ void k_fill_i8(int8_t *p, int64_t n)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace sg

using namespace sg;

extern "C" int sg_fragment_decimate(const sg_instance *inst, const sg_frag_args *args, const uint32_t *thr,
                                    int8_t *spins_out, int32_t *energy_out, void *stream)
{
    if (!inst || !args) return fail(SG_EINVAL, "sg_fragment_decimate: NULL instance or args");
    const int L = inst->L;
    if (!lattice_ok(L)) return fail(SG_EINVAL, "sg_fragment_decimate: L = %d must be even in [4, %d]", L, SG_MAX_L);
    if (!inst->J) return fail(SG_EINVAL, "sg_fragment_decimate: needs the natural-order couplings J");
    if (!thr || !spins_out) return fail(SG_EINVAL, "sg_fragment_decimate: NULL thr or spins");
    const int c = args->core, h = args->halo, l = c + 2 * h;
    if (c < 1 || h < 0 || L % c != 0)
        return fail(SG_EINVAL, "sg_fragment_decimate: core %d must divide L = %d, halo %d >= 0", c, L, h);
    if (l >= L || l > SG_FRAG_MAX_L)
        return fail(SG_EINVAL, "sg_fragment_decimate: fragment edge %d must be < L = %d and <= %d", l, L,
                    SG_FRAG_MAX_L);
    if (args->order != 0 && args->order != 1) return fail(SG_EINVAL, "sg_fragment_decimate: order %d", args->order);
    const int nb = L / c, P = 1 + (h + c - 1) / c;
    if (args->order == 0 && nb % P != 0)
        return fail(SG_EINVAL, "sg_fragment_decimate: colour classes need L/c = %d divisible by %d", nb, P);
    if (args->replicas < 1 || args->replicas > SG_FRAG_MAX_R)
        return fail(SG_EINVAL, "sg_fragment_decimate: replicas = %d outside [1, %d]", args->replicas, SG_FRAG_MAX_R);
    if (args->n_runs < 1 || args->n_sweeps < 1 || args->n_sweeps >= (1 << 30))
        return fail(SG_EINVAL, "sg_fragment_decimate: n_runs = %d, n_sweeps = %d", args->n_runs, args->n_sweeps);
    if (args->K < 1 || args->K > SG_K_MAX) return fail(SG_EINVAL, "sg_fragment_decimate: K = %d", args->K);
    if (static_cast<uint64_t>(args->run0) + static_cast<uint64_t>(args->n_runs) > 0xFFFFFFFFull)
        return fail(SG_ERANGE, "sg_fragment_decimate: run counter words overflow");
    if (static_cast<int64_t>(nb) * nb * nb * args->n_runs > 0x7FFFFFFFll)
        return fail(SG_ERANGE, "sg_fragment_decimate: %d runs of %d cores exceed one launch", args->n_runs,
                    nb * nb * nb);

    FragJob job{};
    job.J = inst->J;
    job.thr = thr;
    job.dec = spins_out;
    job.L = L;
    job.c = c;
    job.h = h;
    job.l = l;
    job.nb = nb;
    job.P = P;
    job.order = args->order;
    job.R = args->replicas;
    job.S = args->n_sweeps;
    job.K = args->K;
    job.run0 = args->run0;
    job.k0 = static_cast<uint32_t>(args->seed);
    job.k1 = static_cast<uint32_t>(args->seed >> 32);
    clear_error();
    hipStream_t st = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    const int64_t total = static_cast<int64_t>(args->n_runs) * L * L * L;
    hipLaunchKernelGGL(k_fill_i8, dim3(static_cast<uint32_t>((total + 255) / 256)), dim3(256), 0, st, spins_out, total);
    const int nq = frag_phases(job);
    for (int q = 0; q < nq; ++q) {
        const int count = frag_phase_count(job, q);
        if (count == 0) continue;
        hipLaunchKernelGGL(k_frag_phase, dim3(static_cast<uint32_t>(count * args->n_runs)),
                           dim3(static_cast<uint32_t>(64 * job.R)), 0, st, job, q, count);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(SG_EDEVICE, "sg_fragment_decimate: launch failed: %s", hipGetErrorString(err));
    if (energy_out) return launch_energy(inst->J, L, args->n_runs, spins_out, energy_out, st);
    return SG_OK;
}
