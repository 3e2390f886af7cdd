// Context creation: validate the RNS primes and build every device table
// once (twiddles, BConv matrices, folded constants; Sec. 5.1 Seq.2).
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <vector>

#include "../../include/ckks_hip.h"
#include "internal.h"

namespace ckks {

namespace {

// --- host modular arithmetic (moduli < 2^32) ---
inline uint64_t mm(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((unsigned __int128)a * b % m); }

uint64_t pw(uint64_t a, uint64_t e, uint64_t m)
{
    uint64_t r = 1 % m;
    a %= m;
    for (; e; e >>= 1, a = mm(a, a, m))
        if (e & 1) r = mm(r, a, m);
    return r;
}

// inverse by the extended Euclidean algorithm
uint64_t inv(uint64_t a, uint64_t m)
{
    int64_t t = 0, nt = 1, r = (int64_t)m, nr = (int64_t)(a % m);
    while (nr) {
        int64_t qq = r / nr, x;
        x = t - qq * nt, t = nt, nt = x;
        x = r - qq * nr, r = nr, nr = x;
    }
    return (uint64_t)(t < 0 ? t + (int64_t)m : t);
}

bool probable_prime(uint64_t n)
{
    if (n < 2) return false;
    for (uint64_t p : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull}) {
        if (n % p == 0) return n == p;
    }
    uint64_t d = n - 1;
    int s = 0;
    while (!(d & 1)) d >>= 1, s++;
    for (uint64_t a : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull}) {
        uint64_t x = pw(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int i = 1; i < s && comp; i++) {
            x = mm(x, x, n);
            if (x == n - 1) comp = false;
        }
        if (comp) return false;
    }
    return true;
}

uint32_t brev(uint32_t x, int bits)
{
    uint32_t r = 0;
    for (int i = 0; i < bits; i++, x >>= 1) r = (r << 1) | (x & 1);
    return r;
}

uint32_t inv32(uint32_t q)  // q^-1 mod 2^32 (q odd), Newton iteration
{
    uint32_t x = q;
    for (int i = 0; i < 5; i++) x *= 2 - q * x;
    return x;
}

// twisted Montgomery pair of constant w mod q
uint2 tw_pair(uint64_t w, uint64_t q, uint32_t qinv)
{
    const uint32_t W = (uint32_t)(((w % q) << 32) % q);
    return make_uint2(W, W * qinv);
}

int32_t centred(uint64_t v, uint64_t q) { return (int32_t)(2 * v < q ? (int64_t)v : (int64_t)v - (int64_t)q); }

// Shoup pair of constant w mod q: (w, floor(w 2^32 / q))
uint2 shoup_pair(uint64_t w, uint64_t q)
{
    w %= q;
    return make_uint2((uint32_t)w, (uint32_t)((w << 32) / q));
}

// constant folded into the last inverse NTT stage: c and c * w1
uint4 fold_pair(uint64_t c, uint64_t w1, uint64_t q)
{
    const uint2 a = shoup_pair(c, q), b = shoup_pair(mm(c, w1, q), q);
    return make_uint4(a.x, a.y, b.x, b.y);
}

}  // namespace

void free_ctx(Ctx* c);

// win_start / win_len (n_win entries, or null for the prefix levels
// 1..n_q): each level is a contiguous window of the ciphertext primes, and
// no two windows have the same number of limbs.
int build_ctx(const ckks_params* p, const int32_t* win_start, const int32_t* win_len, int n_win, Ctx** out)
{
    if (!p || !out) return set_error(CKKS_EINVAL, "null argument");
    if (win_start || win_len) {
        if (!win_start || !win_len || n_win < 1) return set_error(CKKS_EINVAL, "need 1 or more windows");
        bool seen[MAX_PRIMES + 1] = {};
        for (int w = 0; w < n_win; w++) {
            const int st = win_start[w], len = win_len[w];
            if (len < 1 || len > MAX_PRIMES || st < 0 || st > (int)p->n_q - len)
                return set_error(CKKS_EINVAL, "window outside the ciphertext primes");
            if (seen[len]) return set_error(CKKS_EINVAL, "two windows with the same number of limbs");
            seen[len] = true;
        }
    }
    if (p->log_n < 12 || p->log_n > 16) return set_error(CKKS_EUNSUPPORTED, "log_n must be in [12, 16]");
    if (p->n_q < 1 || p->n_p < 1 || p->n_q + p->n_p > MAX_PRIMES)
        return set_error(CKKS_EINVAL, "need 1 <= n_q, 1 <= n_p, n_q + n_p <= 64");
    if (!p->q || !p->p) return set_error(CKKS_EINVAL, "null prime array");
    if (p->n_p > 16) return set_error(CKKS_EUNSUPPORTED, "at most 16 special primes");
    Ctx* c = new (std::nothrow) Ctx();
    if (!c) return set_error(CKKS_EINVAL, "out of host memory");
    c->log_n = (int)p->log_n;
    c->n = 1 << c->log_n;
    c->n_q = (int)p->n_q;
    c->n_p = (int)p->n_p;
    c->n_primes = c->n_q + c->n_p;
    c->dnum = (c->n_q + c->n_p - 1) / c->n_p;
    if (win_start) {
        c->windowed = true;
        for (int l = 0; l <= MAX_PRIMES; l++) c->wbase[l] = -1;
        for (int w = 0; w < n_win; w++) c->wbase[win_len[w]] = win_start[w];
    }
    const uint64_t two_n = 2ull << c->log_n;
    for (int i = 0; i < c->n_primes; i++) {
        const uint64_t m = i < c->n_q ? p->q[i] : p->p[i - c->n_q];
        if (m >= (1ull << 31) || m % two_n != 1 || !probable_prime(m)) {
            delete c;
            return set_error(CKKS_EINVAL, "every prime must be < 2^31, prime and 1 mod 2N");
        }
        for (int k = 0; k < i; k++)
            if (c->mod[k] == m) {
                delete c;
                return set_error(CKKS_EINVAL, "primes must be distinct");
            }
        c->mod[i] = m;
    }
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return set_error(CKKS_EHIP, "no HIP device");
    }

    const int P = c->n_primes, nq = c->n_q, np = c->n_p, N = c->n, L = c->log_n;
    // host images of every table
    std::vector<uint32_t> mods(P), qinvs(P);
    std::vector<uint2> tw_f((size_t)P * N), tw_i((size_t)P * N);
    std::vector<uint32_t> twq_f((size_t)P * N), twq_i((size_t)P * N);
    std::vector<uint4> ninv(P), up_c_r((size_t)(nq + 1) * nq, make_uint4(0, 0, 0, 0));
    std::vector<uint4> up_c((size_t)(nq + 1) * nq, make_uint4(0, 0, 0, 0));
    std::vector<uint64_t> w1(P);  // psi^-brev(1) = psi^-(N/2) per prime
    std::vector<int32_t> up_mat((size_t)(nq + 1) * c->dnum * P * np, 0);
    std::vector<uint4> dn_c(np + nq);
    std::vector<uint2> dn_pinv(nq), rinv(nq), p_r2(nq), rs_qinv((size_t)(nq + 1) * nq, make_uint2(0, 0));
    std::vector<uint2> rs_fin((size_t)(nq + 1) * nq, make_uint2(0, 0));
    std::vector<int32_t> rs_mlast((size_t)nq * np), rs_pr(nq);
    std::vector<int32_t> dn_mat((size_t)nq * np);
    std::vector<uint32_t> p_mod_q(nq);
    std::vector<uint2> r1(P);

    for (int i = 0; i < P; i++) {
        const uint64_t q = c->mod[i];
        mods[i] = (uint32_t)q;
        qinvs[i] = inv32((uint32_t)q);
        // psi: smallest g >= 2 with g^N = -1
        uint64_t psi = 0;
        for (uint64_t g = 2; g < q; g++)
            if (pw(g, (uint64_t)N, q) == q - 1) {
                psi = g;
                break;
            }
        const uint64_t psi_inv = inv(psi, q);
        std::vector<uint64_t> pf(N), pi(N);
        pf[0] = pi[0] = 1;
        for (int e = 1; e < N; e++) pf[e] = mm(pf[e - 1], psi, q), pi[e] = mm(pi[e - 1], psi_inv, q);
        for (int k = 0; k < N; k++) {
            const uint32_t e = brev((uint32_t)k, L);
            tw_f[(size_t)i * N + k] = shoup_pair(pf[e], q);
            tw_i[(size_t)i * N + k] = shoup_pair(pi[e], q);
            twq_f[(size_t)i * N + k] = tw_f[(size_t)i * N + k].y;
            twq_i[(size_t)i * N + k] = tw_i[(size_t)i * N + k].y;
        }
        w1[i] = pi[N / 2];
        ninv[i] = fold_pair(inv((uint64_t)N, q), w1[i], q);
    }
    const auto R = [&](int i) { return (1ull << 32) % c->mod[i]; };  // 2^32 mod prime i

    // ModUp constants per level and digit (prime ids lo..hi-1 of key digit jk)
    for (int level = 1; level <= nq; level++) {
        if (!c->has_level(level)) continue;
        for (int j = 0; j < c->digits(level); j++) {
            const int lo = c->wbase[level] + c->digit_lo(j, level), hi = c->wbase[level] + c->digit_hi(j, level);
            const int jk = c->key_digit(j, level);
            for (int i = lo; i < hi; i++) {
                const uint64_t q = c->mod[i];
                uint64_t dh = 1;
                for (int s = lo; s < hi; s++)
                    if (s != i) dh = mm(dh, c->mod[s], q);
                const uint64_t base = mm(inv((uint64_t)N, q), inv(dh, q), q);
                up_c[(size_t)level * nq + i] = fold_pair(base, w1[i], q);
                up_c_r[(size_t)level * nq + i] = fold_pair(mm(base, R(i), q), w1[i], q);
            }
            for (int t = 0; t < P; t++) {
                const uint64_t qt = c->mod[t];
                for (int s = lo; s < hi; s++) {
                    uint64_t dh = 1;
                    for (int r = lo; r < hi; r++)
                        if (r != s) dh = mm(dh, c->mod[r], qt);
                    up_mat[(((size_t)level * c->dnum + jk) * P + t) * np + (s - lo)] = centred(dh, qt);
                }
            }
        }
    }
    // ModDown constants
    for (int k = 0; k < np; k++) {
        const uint64_t pk = c->mod[nq + k];
        uint64_t ph = 1;
        for (int r = 0; r < np; r++)
            if (r != k) ph = mm(ph, c->mod[nq + r], pk);
        const uint64_t r2 = mm(R(nq + k), R(nq + k), pk);
        dn_c[k] = fold_pair(mm(mm(inv((uint64_t)N, pk), inv(ph, pk), pk), r2, pk), w1[nq + k], pk);
    }
    for (int i = 0; i < nq; i++) {
        const uint64_t q = c->mod[i];
        uint64_t pp = 1;
        for (int k = 0; k < np; k++) pp = mm(pp, c->mod[nq + k], q);
        const uint64_t rinv_q = inv(R(i), q), r2 = mm(R(i), R(i), q);
        for (int k = 0; k < np; k++) {
            uint64_t ph = 1;
            for (int r = 0; r < np; r++)
                if (r != k) ph = mm(ph, c->mod[nq + r], q);
            dn_mat[(size_t)i * np + k] = centred(mm(ph, rinv_q, q), q);
        }
        dn_pinv[i] = tw_pair(mm(inv(pp, q), r2, q), q, qinvs[i]);
        // fused rescale when q_i is the dropped prime
        dn_c[np + i] = fold_pair(mm(mm(inv((uint64_t)N, q), r2, q), inv(pp, q), q), w1[i], q);
        for (int k = 0; k < np; k++) {
            uint64_t ph = 1;
            for (int r = 0; r < np; r++)
                if (r != k) ph = mm(ph, c->mod[nq + r], q);
            rs_mlast[(size_t)i * np + k] = centred(mm(mm(ph, inv(pp, q), q), R(i), q), q);
        }
        rs_pr[i] = centred(mm(pp, rinv_q, q), q);
        p_mod_q[i] = (uint32_t)pp;
        rinv[i] = tw_pair(rinv_q, q, qinvs[i]);
        p_r2[i] = tw_pair(mm(pp, mm(rinv_q, rinv_q, q), q), q, qinvs[i]);
    }
    // rescale: [q_{l-1}^-1]_{q_i}
    for (int level = 2; level <= nq; level++)
        for (int i = 0; i < level - 1; i++)
        {
            const uint64_t q = c->mod[i];
            uint64_t pp = 1;
            for (int k = 0; k < np; k++) pp = mm(pp, c->mod[nq + k], q);
            const uint64_t qlinv = inv(c->mod[level - 1] % q, q);
            rs_qinv[(size_t)level * nq + i] = tw_pair(qlinv, q, qinvs[i]);
            rs_fin[(size_t)level * nq + i] = tw_pair(mm(mm(inv(pp, q), qlinv, q), mm(R(i), R(i), q), q), q, qinvs[i]);
        }

    for (int i = 0; i < P; i++) r1[i] = tw_pair(R(i), c->mod[i], qinvs[i]);

    // merged ModDown + rational rescaling, per window with a window below
    std::vector<uint4> rr_c, rr2_c;
    std::vector<int32_t> rr_mat, rr2_mat;
    std::vector<uint2> rr_fin, rr2_fin;
    for (int level = 1; level <= nq && c->windowed; level++) {
        if (!c->has_level(level)) continue;
        int below = 0;
        for (int l = level - 1; l >= 1 && !below; l--)
            if (c->has_level(l)) below = l;
        if (!below) continue;
        const int b = c->wbase[level], b2 = c->wbase[below];
        const int klo = b > b2 ? b : b2, khi = b + level < b2 + below ? b + level : b2 + below;
        c->rr_below[level] = below;
        c->rr_dlo[level] = klo - b;
        c->rr_dhi[level] = khi - b > klo - b ? khi - b : klo - b;
        // S = P, then the dropped window rows in slot order
        std::vector<int> S;
        for (int k = 0; k < np; k++) S.push_back(nq + k);
        for (int r = 0; r < level; r++)
            if (r < c->rr_dlo[level] || r >= c->rr_dhi[level]) S.push_back(b + r);
        auto kept = [&](int pid) { return pid >= b && pid < b + level; };  // output prime also in the window
        c->rr_c_off[level] = (int)rr_c.size();
        c->rr_mat_off[level] = (int)rr_mat.size();
        c->rr_fin_off[level] = (int)rr_fin.size();
        for (int s : S) {
            const uint64_t q = c->mod[s];
            uint64_t sh = 1, qa = 1;
            for (int t : S)
                if (t != s) sh = mm(sh, c->mod[t] % q, q);
            for (int o = 0; o < below; o++)
                if (!kept(b2 + o)) qa = mm(qa, c->mod[b2 + o] % q, q);
            const uint64_t r2 = mm(R(s), R(s), q);
            rr_c.push_back(fold_pair(mm(mm(inv((uint64_t)N, q), inv(sh, q), q), mm(r2, qa, q), q), w1[s], q));
        }
        for (int o = 0; o < below; o++) {
            const int pid = b2 + o;
            const uint64_t q = c->mod[pid];
            uint64_t qa = 1, qs = 1;
            for (int a = 0; a < below; a++)
                if (!kept(b2 + a)) qa = mm(qa, c->mod[b2 + a] % q, q);
            for (int t : S) qs = mm(qs, c->mod[t] % q, q);
            const uint64_t rinv_q = inv(R(pid), q), f = kept(pid) ? inv(qa, q) : 1;
            for (int s : S) {
                uint64_t sh = 1;
                for (int t : S)
                    if (t != s) sh = mm(sh, c->mod[t] % q, q);
                rr_mat.push_back(centred(mm(mm(sh, rinv_q, q), f, q), q));
            }
            const uint64_t fin = mm(mm(kept(pid) ? qa : 1, inv(qs, q), q), mm(R(pid), R(pid), q), q);
            rr_fin.push_back(tw_pair(fin, q, qinvs[pid]));
        }
        // stand-alone rational rescaling: S = D (the dropped window rows)
        const std::vector<int> D(S.begin() + np, S.end());
        c->rr2_c_off[level] = (int)rr2_c.size();
        c->rr2_mat_off[level] = (int)rr2_mat.size();
        c->rr2_fin_off[level] = (int)rr2_fin.size();
        for (int d : D) {
            const uint64_t q = c->mod[d];
            uint64_t dh = 1, qa = 1;
            for (int t : D)
                if (t != d) dh = mm(dh, c->mod[t] % q, q);
            for (int o = 0; o < below; o++)
                if (!kept(b2 + o)) qa = mm(qa, c->mod[b2 + o] % q, q);
            rr2_c.push_back(fold_pair(mm(mm(inv((uint64_t)N, q), inv(dh, q), q), qa, q), w1[d], q));
        }
        for (int o = 0; o < below; o++) {
            const int pid = b2 + o;
            const uint64_t q = c->mod[pid];
            uint64_t qa = 1, qd = 1;
            for (int a = 0; a < below; a++)
                if (!kept(b2 + a)) qa = mm(qa, c->mod[b2 + a] % q, q);
            for (int t : D) qd = mm(qd, c->mod[t] % q, q);
            const uint64_t f = kept(pid) ? inv(qa, q) : 1;
            for (int d : D) {
                uint64_t dh = 1;
                for (int t : D)
                    if (t != d) dh = mm(dh, c->mod[t] % q, q);
                rr2_mat.push_back(centred(mm(mm(dh, R(pid), q), f, q), q));
            }
            rr2_fin.push_back(tw_pair(mm(kept(pid) ? qa : 1, inv(qd, q), q), q, qinvs[pid]));
        }
    }
    if (rr_c.empty()) rr_c.push_back(make_uint4(0, 0, 0, 0));
    if (rr_mat.empty()) rr_mat.push_back(0);
    if (rr_fin.empty()) rr_fin.push_back(make_uint2(0, 0));
    if (rr2_c.empty()) rr2_c.push_back(make_uint4(0, 0, 0, 0));
    if (rr2_mat.empty()) rr2_mat.push_back(0);
    if (rr2_fin.empty()) rr2_fin.push_back(make_uint2(0, 0));
    for (std::vector<int32_t>* m : {&up_mat, &dn_mat, &rs_mlast, &rr_mat, &rr2_mat}) m->resize(m->size() + BCONV_MAT_PAD, 0);
    std::vector<int32_t> lv_tab(4 * (MAX_PRIMES + 1), 0);
    for (int l = 0; l <= MAX_PRIMES; l++) {
        const bool ok = c->windowed && l >= 1 && l <= nq && c->has_level(l);
        lv_tab[l] = c->windowed ? (ok ? c->wbase[l] : -1) : 0;
        lv_tab[(MAX_PRIMES + 1) + l] = ok && c->rr_below[l] ? c->rr_drop(l) : 0;
        lv_tab[2 * (MAX_PRIMES + 1) + l] = ok ? c->rr_dlo[l] : 0;
        lv_tab[3 * (MAX_PRIMES + 1) + l] = ok ? c->rr_dhi[l] : 0;
    }

    // one device block, 256-byte aligned pieces
    struct Piece {
        void** dst;
        const void* src;
        size_t bytes;
    };
    std::vector<Piece> pieces = {
        {(void**)&c->mods, mods.data(), mods.size() * 4},
        {(void**)&c->qinvs, qinvs.data(), qinvs.size() * 4},
        {(void**)&c->tw_fwd, tw_f.data(), tw_f.size() * 8},
        {(void**)&c->tw_inv, tw_i.data(), tw_i.size() * 8},
        {(void**)&c->twq_fwd, twq_f.data(), twq_f.size() * 4},
        {(void**)&c->twq_inv, twq_i.data(), twq_i.size() * 4},
        {(void**)&c->ninv, ninv.data(), ninv.size() * 16},
        {(void**)&c->up_c_r, up_c_r.data(), up_c_r.size() * 16},
        {(void**)&c->up_c, up_c.data(), up_c.size() * 16},
        {(void**)&c->up_mat, up_mat.data(), up_mat.size() * 4},
        {(void**)&c->dn_c, dn_c.data(), dn_c.size() * 16},
        {(void**)&c->dn_mat, dn_mat.data(), dn_mat.size() * 4},
        {(void**)&c->dn_pinv, dn_pinv.data(), dn_pinv.size() * 8},
        {(void**)&c->p_mod_q, p_mod_q.data(), p_mod_q.size() * 4},
        {(void**)&c->rinv, rinv.data(), rinv.size() * 8},
        {(void**)&c->p_r2, p_r2.data(), p_r2.size() * 8},
        {(void**)&c->r1, r1.data(), r1.size() * 8},
        {(void**)&c->rs_qinv, rs_qinv.data(), rs_qinv.size() * 8},
        {(void**)&c->rs_mlast, rs_mlast.data(), rs_mlast.size() * 4},
        {(void**)&c->rs_pr, rs_pr.data(), rs_pr.size() * 4},
        {(void**)&c->rs_fin, rs_fin.data(), rs_fin.size() * 8},
        {(void**)&c->rr_c, rr_c.data(), rr_c.size() * 16},
        {(void**)&c->rr_mat, rr_mat.data(), rr_mat.size() * 4},
        {(void**)&c->rr_fin, rr_fin.data(), rr_fin.size() * 8},
        {(void**)&c->rr2_c, rr2_c.data(), rr2_c.size() * 16},
        {(void**)&c->rr2_mat, rr2_mat.data(), rr2_mat.size() * 4},
        {(void**)&c->rr2_fin, rr2_fin.data(), rr2_fin.size() * 8},
        {(void**)&c->lv_tab, lv_tab.data(), lv_tab.size() * 4},
    };
    size_t total = 0;
    for (auto& pc : pieces) total += (pc.bytes + 255) & ~(size_t)255;
    if (hipMalloc(&c->dev_block, total) != hipSuccess) {
        delete c;
        return set_error(CKKS_EHIP, "hipMalloc of context tables failed");
    }
    c->dev_bytes = total;
    std::vector<char> host(total, 0);
    size_t off = 0;
    for (auto& pc : pieces) {
        std::memcpy(host.data() + off, pc.src, pc.bytes);
        *pc.dst = static_cast<char*>(c->dev_block) + off;
        off += (pc.bytes + 255) & ~(size_t)255;
    }
    if (hipMemcpy(c->dev_block, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(c->dev_block);
        delete c;
        return set_error(CKKS_EHIP, "uploading context tables failed");
    }
    if (int e = build_plans(*c)) {
        free_ctx(c);
        return e;
    }
    *out = c;
    return CKKS_OK;
}

void free_ctx(Ctx* c)
{
    if (!c) return;
    if (c->dev_block) (void)hipFree(c->dev_block);
    if (c->plan_block) (void)hipFree(c->plan_block);
    if (c->dir_block) (void)hipFree(c->dir_block);
    delete c;
}

// Constants of the stand-alone base conversion (the values the device set-up
// kernel computes): cs[s] = twisted [Shat_s^-1]_{q_s}; ms[t n_in + s] =
// centred [Shat_s 2^32]_{q_t}.
void bconv_consts(const Ctx& c, const int32_t* in_ids, int n_in, const int32_t* out_ids, int n_out, uint2* cs,
                  int32_t* ms)
{
    for (int s = 0; s < n_in; s++) {
        const uint64_t qs = c.mod[in_ids[s]];
        uint64_t prod = 1;
        for (int r = 0; r < n_in; r++)
            if (r != s) prod = mm(prod, c.mod[in_ids[r]] % qs, qs);
        cs[s] = tw_pair(inv(prod, qs), qs, inv32((uint32_t)qs));
    }
    for (int t = 0; t < n_out; t++) {
        const uint64_t qt = c.mod[out_ids[t]];
        for (int s = 0; s < n_in; s++) {
            uint64_t prod = 1;
            for (int r = 0; r < n_in; r++)
                if (r != s) prod = mm(prod, c.mod[in_ids[r]] % qt, qt);
            ms[t * n_in + s] = centred(mm(prod, (1ull << 32) % qt, qt), qt);
        }
    }
}

// ---------------------------------------------------------------------------
// Rational rescaling (25-30 prime system): from the primes in_ids to out_ids,
// D = dropped, A = added, K = kept.  Host side computes the exact constants;
// the device runs
//   y_d = x_d * Q_A  (d in D)                      [lincomb]
//   INTT(y), conv = BConv_{D -> out}(y), NTT(conv)   [existing passes]
//   out_o = x_o * Q_A Q_D^-1 - conv_o * Q_D^-1     [lincomb; x_o = 0 for o in A]
// Workspace: y [2][|D|][N], conv [2][n_out][N], BConv scratch.
// ---------------------------------------------------------------------------
size_t rescale_rational_ws_bytes(const Ctx& c, int n_in, int n_out)
{
    const size_t n = c.n;  // generic path: 2 n_in + 2 n_out rows; window path: 4 dropped + 2 n_out rows
    return 4 * n * (4 * (size_t)n_in + 2 * (size_t)n_out) + bconv_ws_bytes(c, n_in, n_out);
}

int launch_rescale_rational(const Ctx& c, const uint32_t* ct, int n_in, const int32_t* in_ids, int n_out,
                            const int32_t* out_ids, uint32_t* out, void* ws, hipStream_t s)
{
    // a windowed context's transition to the window below: precomputed plan
    if (c.windowed && c.has_level(n_in) && c.rr_below[n_in] == n_out) {
        bool match = true;
        for (int i = 0; i < n_in; i++) match &= in_ids[i] == c.wbase[n_in] + i;
        for (int o = 0; o < n_out; o++) match &= out_ids[o] == c.wbase[n_out] + o;
        if (match) return launch_rescale_rational_window(c, n_in, ct, out, ws, s);
    }
    const size_t n = c.n;
    int32_t drop[MAX_PRIMES], dpos[MAX_PRIMES], kpos[MAX_PRIMES];
    int nd = 0;
    for (int i = 0; i < n_in; i++) {
        bool kept = false;
        for (int o = 0; o < n_out; o++) kept |= out_ids[o] == in_ids[i];
        if (!kept) drop[nd] = in_ids[i], dpos[nd++] = i;
    }
    for (int o = 0; o < n_out; o++) {
        kpos[o] = -1;
        for (int i = 0; i < n_in; i++)
            if (in_ids[i] == out_ids[o]) kpos[o] = i;
    }
    if (nd == 0) return set_error(CKKS_EINVAL, "rational rescaling drops no prime");
    uint32_t* y = static_cast<uint32_t*>(ws);              // [2][nd][N]
    uint32_t* conv = y + 2 * (size_t)nd * n;                // [2][n_out][N]
    void* bws = conv + 2 * (size_t)n_out * n;
    // y_d = x_d * Q_A mod d
    LincombArgs L{};
    L.n = nd;
    for (int k = 0; k < nd; k++) {
        const uint64_t d = c.mod[drop[k]];
        uint64_t qa = 1;
        for (int o = 0; o < n_out; o++)
            if (kpos[o] < 0) qa = mm(qa, c.mod[out_ids[o]] % d, d);
        L.xrow[k] = dpos[k];
        L.q[k] = (uint32_t)d;
        L.a[k] = tw_pair(qa, d, inv32((uint32_t)d));
    }
    if (int e = launch_lincomb(c, L, ct, (size_t)n_in * n, nullptr, 0, y, (size_t)nd * n, s)) return e;
    int32_t ids2[2 * MAX_PRIMES];
    for (int k = 0; k < nd; k++) ids2[k] = ids2[nd + k] = drop[k];
    if (int e = launch_ntt(c, true, y, ids2, 2 * nd, s)) return e;
    for (int h = 0; h < 2; h++)
        if (int e = launch_bconv(c, y + (size_t)h * nd * n, drop, nd, conv + (size_t)h * n_out * n, out_ids, n_out,
                                 bws, s))
            return e;
    for (int o = 0; o < n_out; o++) ids2[o] = ids2[n_out + o] = out_ids[o];
    if (int e = launch_ntt(c, false, conv, ids2, 2 * n_out, s)) return e;
    // out_o = x_o * Q_A Q_D^-1 - conv_o * Q_D^-1
    L = LincombArgs{};
    L.n = n_out;
    for (int o = 0; o < n_out; o++) {
        const uint64_t m = c.mod[out_ids[o]];
        uint64_t qa = 1, qd = 1;
        for (int p = 0; p < n_out; p++)
            if (kpos[p] < 0) qa = mm(qa, c.mod[out_ids[p]] % m, m);
        for (int k = 0; k < nd; k++) qd = mm(qd, c.mod[drop[k]] % m, m);
        const uint64_t qdi = inv(qd, m);
        const uint32_t qinv = inv32((uint32_t)m);
        L.xrow[o] = kpos[o];
        L.q[o] = (uint32_t)m;
        L.a[o] = tw_pair(mm(qa, qdi, m), m, qinv);
        L.b[o] = tw_pair((m - qdi) % m, m, qinv);
    }
    return launch_lincomb(c, L, ct, (size_t)n_in * n, conv, (size_t)n_out * n, out, (size_t)n_out * n, s);
}

// The `count` largest primes below 2^bits that are 1 mod 2N, descending.
int prime_chain(int bits, int log_n, int count, uint64_t* out)
{
    if (bits < 2 || bits > 32 || log_n < 1 || log_n > 20 || count < 0 || (!out && count))
        return set_error(CKKS_EINVAL, "bad prime_chain arguments");
    const uint64_t step = 2ull << log_n;
    uint64_t cand = (((1ull << bits) - 2) / step) * step + 1;
    int got = 0;
    while (got < count && cand > step) {
        if (probable_prime(cand)) out[got++] = cand;
        cand -= step;
    }
    return got == count ? CKKS_OK : set_error(CKKS_EINVAL, "not enough primes of that size");
}

}  // namespace ckks
