// The three-party protocol of the paper (Sec. III-B, initialization and
// recommendation phases) around the encrypted MF program, with every message
// between the parties serialised and counted.
//
// Parties: the users, the recommendation server (RS) and the crypto service
// provider (CSP, the key holder).  One context plays all three; a message is
// a ciphertext exported to coefficient form (8 bytes per residue, both
// polynomials, limbs q_0..q_level) and imported on the other side, or a
// vector of doubles.  Channels:
//   0 CSP -> users   public key (one copy per user)
//   1 CSP -> RS      public key and evaluation keys (relinearisation, rotations)
//   2 users -> RS    each user's encrypted ratings (its row, one rating per slot)
//   3 RS -> CSP      the same ciphertexts with the RS's masks added
//   4 CSP -> RS      the masked ratings re-packed in the CSR block layout and
//                    encrypted anew (the rating ciphertexts of the MF program)
//   5 RS -> CSP      masked encrypted predictions
//   6 CSP -> users   masked plaintext predictions (doubles)
//   7 RS -> users    the prediction masks (doubles), which only the RS and the
//                    users know
// The paper counts ciphertexts CSP -> RS and RS -> users as (1 + M/L) with one
// rating per slot; the block layout here holds D = N/(2B) ratings per
// ciphertext (a rating occupies the B slots of its block), so channel 4
// carries ceil-by-packing(M / D) ciphertexts.
//
// Masks: the RS draws a real mask per rating from ChaCha20 (purpose 12, object
// = rating index, limb 0): m = ((w mod 2^21) - 2^20) / 2^10, in [-1024, 1024)
// with 2^-10 steps, added to the encrypted rating as a plaintext and removed
// from the re-packed ciphertexts by subtracting the same values in the block
// layout; prediction masks use purpose 13 the same way.
#include <cmath>
#include <cstring>

#include "host_math.h"
#include "mf_internal.h"

namespace csrmf {

namespace {

constexpr uint32_t kRatingMask = 12, kPredMask = 13;
constexpr uint32_t kUserSerial = 0x50000000u;    // + user index * 64 + chunk: the users' encryptions
constexpr uint32_t kCspSerial = 0x58000000u;     // + rating ciphertext index: the CSP's re-encryption

double mask_value(const uint8_t seed[32], uint32_t purpose, uint32_t obj) {
    uint64_t w;
    chacha20_words(seed, purpose, obj, 0, 1, &w);
    return (double)((int64_t)(w % (1ull << 21)) - (1ll << 20)) / 1024.0;
}

size_t ct_bytes(const Context* c, int level) { return 2 * (size_t)(level + 1) * c->N * 8; }

// a ciphertext crossing a channel: exported, counted, imported by the receiver
Ct send(Context* c, ProtocolCounters& k, int ch, const Ct& x) {
    std::vector<uint64_t> buf(2 * (size_t)(x.level + 1) * c->N);
    c->export_ct(x, buf.data());
    k.msgs[ch] += 1;
    k.bytes[ch] += (int64_t)(buf.size() * 8);
    return c->import_ct(buf.data(), x.level, x.scale);
}

void decrypt_values(Context* c, const Ct& x, std::vector<double>& z) {
    std::vector<int64_t> m(c->N);
    c->decrypt_int(x, m.data());
    z.assign(c->N / 2, 0.0);
    ckks_decode(m.data(), c->logN, x.scale, z.data(), (int)(c->N / 2));
}

}  // namespace

void protocol_ingest(Context* c, int32_t n_rows, int32_t n_cols, const int64_t* row_ptr, const int32_t* col_idx,
                     const double* values) {
    if (!c->have_keys) throw Error(CSRMF_E_STATE, "keygen first (the CSP's key pair)");
    if (!values) throw Error(CSRMF_E_INVAL, "values");
    mfp::install_layout(c, n_rows, n_cols, row_ptr, col_idx);   // also the program's rotation keys
    MfState& m = *c->mf;
    ProtocolCounters& k = c->proto;
    k = ProtocolCounters();
    const int L = c->L;
    const double scale = std::ldexp(1.0, c->prm.log2_scale);
    const size_t half = c->N / 2;
    // initialization: the CSP hands out the public key (and the RS's evaluation keys)
    const int64_t pk_bytes = (int64_t)ct_bytes(c, L);
    const int64_t key_bytes = (int64_t)(2 * (size_t)(L + 1 + c->alpha) * c->N * 8);
    k.msgs[0] += n_rows;
    k.bytes[0] += pk_bytes * n_rows;
    k.msgs[1] += 1 + 1 + (int64_t)c->rot.size();
    k.bytes[1] += pk_bytes + key_bytes * (int64_t)c->relin.n_digits * (1 + (int64_t)c->rot.size());
    // users encrypt their rows (one rating per slot), RS masks them, CSP
    // decrypts the masked values
    std::vector<double> masked(m.nnz);
    std::vector<double> z(half);
    std::vector<int64_t> pt(c->N);
    for (int i = 0; i < n_rows; ++i) {
        for (int64_t s = row_ptr[i]; s < row_ptr[i + 1]; s += (int64_t)half) {
            const int64_t e = std::min<int64_t>(row_ptr[i + 1], s + (int64_t)half);
            const uint32_t chunk = (uint32_t)((s - row_ptr[i]) / (int64_t)half);
            std::fill(z.begin(), z.end(), 0.0);
            for (int64_t p = s; p < e; ++p) z[p - s] = values[p];
            if (!ckks_encode(z.data(), (int)half, c->logN, scale, pt.data()))
                throw Error(CSRMF_E_INVAL, "rating too large to encode");
            std::vector<Ct> enc;
            const uint32_t ser = kUserSerial + (uint32_t)i * 64u + chunk;
            c->encrypt_int_batch(pt.data(), 1, L, scale, enc, &ser);                       // user i
            Ct at_rs = send(c, k, 2, enc[0]);                                             // users -> RS
            c->pool.put(enc[0].d);
            std::fill(z.begin(), z.end(), 0.0);
            for (int64_t p = s; p < e; ++p) z[p - s] = mask_value(c->seed, kRatingMask, (uint32_t)p);
            ckks_encode(z.data(), (int)half, c->logN, scale, pt.data());
            Ct mk;
            c->add_plain(at_rs, pt.data(), mk);                                           // RS masks
            c->pool.put(at_rs.d);
            Ct at_csp = send(c, k, 3, mk);                                                // RS -> CSP
            c->pool.put(mk.d);
            std::vector<double> dz;
            decrypt_values(c, at_csp, dz);                                                // CSP
            c->pool.put(at_csp.d);
            for (int64_t p = s; p < e; ++p) masked[p] = dz[p - s];
        }
    }
    // the CSP re-packs the masked ratings in the CSR block layout and encrypts them
    std::vector<std::vector<double>> zs(m.n_ct, std::vector<double>(half));
    mfp::fill_rating_slots(m, 0, masked.data(), nullptr, nullptr, zs);
    std::vector<int64_t> pts = mfp::encode_all(c, zs, scale);
    std::vector<uint32_t> sers(m.n_ct);
    for (int t = 0; t < m.n_ct; ++t) sers[t] = kCspSerial + (uint32_t)t;
    std::vector<Ct> R;
    c->encrypt_int_batch(pts.data(), m.n_ct, L, scale, R, sers.data());
    // the RS receives them and removes its masks in the same layout
    std::vector<double> mvals(m.nnz);
    for (int p = 0; p < m.nnz; ++p) mvals[p] = mask_value(c->seed, kRatingMask, (uint32_t)p);
    mfp::fill_rating_slots(m, 0, mvals.data(), nullptr, nullptr, zs);
    std::vector<int64_t> mpts = mfp::encode_all(c, zs, scale);
    std::vector<uint64_t> handles;
    for (int t = 0; t < m.n_ct; ++t) {
        Ct at_rs = send(c, k, 4, R[t]);                                                   // CSP -> RS
        c->pool.put(R[t].d);
        std::vector<int64_t> neg(c->N);
        for (uint64_t n = 0; n < c->N; ++n) neg[n] = -mpts[(size_t)t * c->N + n];
        Ct clean;
        c->add_plain(at_rs, neg.data(), clean);                                           // RS unmasks
        c->pool.put(at_rs.d);
        handles.push_back(c->put(clean));
    }
    m.R = handles;
    c->sync();
}

void protocol_recommend(Context* c, int which, double* rhat) {
    MfState& m = mfp::state(c);
    const std::vector<uint64_t>& src = which == 0 ? m.Sdot : m.Pred;
    if (src.empty()) throw Error(CSRMF_E_STATE, which == 0 ? "no epoch has run" : "csrmf_predict has not run");
    ProtocolCounters& k = c->proto;
    const size_t half = c->N / 2;
    // RS masks each prediction slot tB of the rating layout
    std::vector<double> pm(m.nnz);
    for (int p = 0; p < m.nnz; ++p) pm[p] = mask_value(c->seed, kPredMask, (uint32_t)p);
    std::vector<std::vector<double>> zs(m.n_ct, std::vector<double>(half, 0.0));
    for (int r = 0; r < m.nnz; ++r) zs[m.ct_of[r]][(size_t)m.blk_of[r] * m.B] = pm[r];
    std::vector<double> masked(m.nnz);
    std::vector<int64_t> pt(c->N);
    for (int t = 0; t < m.n_ct; ++t) {
        const Ct& s = c->get(src[t]);
        if (!ckks_encode(zs[t].data(), (int)half, c->logN, s.scale, pt.data()))
            throw Error(CSRMF_E_INVAL, "prediction mask too large to encode");
        Ct mk;
        c->add_plain(s, pt.data(), mk);                                                   // RS masks
        Ct at_csp = send(c, k, 5, mk);                                                    // RS -> CSP
        c->pool.put(mk.d);
        std::vector<double> z;
        decrypt_values(c, at_csp, z);                                                     // CSP
        c->pool.put(at_csp.d);
        for (int r = 0; r < m.nnz; ++r)
            if (m.ct_of[r] == t) masked[r] = z[(size_t)m.blk_of[r] * m.B];
    }
    // CSP -> users: masked plaintext predictions; RS -> users: the masks (doubles)
    for (int i = 0; i < m.n_users; ++i) {
        const int64_t d = m.row_ptr[i + 1] - m.row_ptr[i];
        if (!d) continue;
        k.msgs[6] += 1;
        k.bytes[6] += d * 8;
        k.msgs[7] += 1;
        k.bytes[7] += d * 8;
    }
    for (int r = 0; r < m.nnz; ++r) rhat[r] = masked[r] - pm[r];                         // users unmask
}

}  // namespace csrmf

using csrmf::Context;
using csrmf::Error;

extern "C" {

int csrmf_protocol_ingest(csrmf_ctx* cx, int32_t n_rows, int32_t n_cols, const int64_t* row_ptr,
                          const int32_t* col_idx, const double* values, int32_t* n_ct) {
    Context* c = reinterpret_cast<Context*>(cx);
    if (!c) {
        csrmf::last_error() = "null context";
        return CSRMF_E_INVAL;
    }
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    try {
        csrmf::protocol_ingest(c, n_rows, n_cols, row_ptr, col_idx, values);
        if (n_ct) *n_ct = c->mf->n_ct;
        csrmf::last_error().clear();
        return CSRMF_OK;
    } catch (const Error& e) {
        csrmf::last_error() = e.what();
        return e.code;
    } catch (const std::exception& e) {
        csrmf::last_error() = e.what();
        return CSRMF_E_DEVICE;
    }
}

int csrmf_protocol_recommend(csrmf_ctx* cx, int32_t which, double* rhat) {
    Context* c = reinterpret_cast<Context*>(cx);
    if (!c || !rhat || (which != 0 && which != 1)) {
        csrmf::last_error() = "protocol_recommend: bad arguments";
        return CSRMF_E_INVAL;
    }
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    try {
        csrmf::protocol_recommend(c, which, rhat);
        csrmf::last_error().clear();
        return CSRMF_OK;
    } catch (const Error& e) {
        csrmf::last_error() = e.what();
        return e.code;
    } catch (const std::exception& e) {
        csrmf::last_error() = e.what();
        return CSRMF_E_DEVICE;
    }
}

int csrmf_protocol_counters(const csrmf_ctx* cx, int64_t* msgs, int64_t* bytes) {
    const Context* c = reinterpret_cast<const Context*>(cx);
    if (!c || !msgs || !bytes) {
        csrmf::last_error() = "protocol_counters: null argument";
        return CSRMF_E_INVAL;
    }
    for (int i = 0; i < csrmf::ProtocolCounters::kChannels; ++i) {
        msgs[i] = c->proto.msgs[i];
        bytes[i] = c->proto.bytes[i];
    }
    return CSRMF_OK;
}

}  // extern "C"
