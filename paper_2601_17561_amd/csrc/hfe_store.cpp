// Saving and loading an encrypted database.  The database is the artefact the method prepares
// once and keeps (Section 6.3: the encrypted database is stored and stays resident; its size is the
// scheme's main storage cost), so a server restarts by reading it back instead of encrypting it
// again.  The file holds a header, a fingerprint of the keys it was written under, and the device
// buffers of every prepared form, streamed through a small pinned staging buffer so that host memory
// stays bounded whatever the database size.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>

#include "hfe_internal.h"

using namespace hfe;

namespace {

constexpr char kMagic[8] = {'H', 'F', 'E', 'D', 'B', 'v', '0', '1'};
constexpr size_t kStage = 64ull << 20;  // pinned staging buffer

struct FileHeader {
  char magic[8];
  uint64_t key_print;                      // fingerprint of the keys (parameters and secrets)
  int64_t d1, R, K, KB, R_pad;
  uint32_t forms;
  int32_t n_rns, n_p2, n_primes;
  uint64_t bytes[4];                       // plain residues, digit planes, RNS planes, n^2 planes
};

// FNV-1a over a byte range (a fingerprint against mixing up keys, not a security property).
uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 0x100000001b3ull;
  return h;
}
template <class T>
uint64_t fnv1a_v(uint64_t h, T v) {
  return fnv1a(h, &v, sizeof(v));
}

// Every parameter field (not the struct bytes, whose padding is unspecified) and both secrets.
uint64_t key_print(const hfe_keys* K) {
  const hfe_params& P = K->P;
  uint64_t h = 0xcbf29ce484222325ull;
  h = fnv1a_v(h, P.log_n_db);
  h = fnv1a_v(h, P.log_n_q);
  h = fnv1a_v(h, P.n_q_primes);
  for (uint32_t i = 0; i < P.n_q_primes && i < HFE_MAX_QPRIMES; ++i) h = fnv1a_v(h, P.q[i]);
  h = fnv1a_v(h, P.p);
  h = fnv1a_v(h, P.gap_bits);
  h = fnv1a_v(h, P.d2);
  h = fnv1a_v(h, P.max_db_rows);
  h = fnv1a(h, K->s_host.data(), K->s_host.size());
  h = fnv1a(h, K->sdb_host.data(), K->sdb_host.size());
  return h;
}

struct Pinned {
  void* p = nullptr;
  ~Pinned() {
    if (p) (void)hipHostFree(p);
  }
};

struct File {
  FILE* f = nullptr;
  ~File() {
    if (f) std::fclose(f);
  }
};

// The device buffers of a database in file order, with their expected sizes.
void expected_bytes(const hfe_db* D, uint64_t out[4]) {
  const size_t np = (size_t)D->slots_planes;
  const size_t plane = (size_t)D->KB * D->R_pad * kKB;
  out[0] = (D->forms & HFE_FORM_PLAIN_U64) ? sizeof(uint64_t) * (size_t)D->slots_plain * D->K * D->R : 0;
  out[1] = (D->forms & HFE_FORM_I8_MFMA) ? np * kDigits * plane : 0;
  out[2] = (D->forms & HFE_FORM_RNS_I8) ? np * D->n_rns * plane : 0;
  out[3] = (D->forms & HFE_FORM_P2_I8) ? np * 2 * D->n_p2 * plane : 0;
}

}  // namespace

extern "C" {

hfe_status hfe_db_save(const hfe_db* db, const char* path, void* stream) {
  const HandleBase* hb = static_cast<const HandleBase*>(static_cast<const void*>(db));
  if (!db || hb->kind != kDb) return fail(HFE_EINVAL, "invalid database handle");
  if (!path) return fail(HFE_EINVAL, "path is NULL");
  if (db->keys->family != 0) return fail(HFE_EINVAL, "databases of the n^2 modulus chain are not stored");
  const hipStream_t s = (hipStream_t)stream;
  FileHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kMagic, sizeof(kMagic));
  h.key_print = key_print(db->keys);
  h.d1 = db->d1;
  h.R = db->R;
  h.K = db->K;
  h.KB = db->KB;
  h.R_pad = db->R_pad;
  h.forms = db->forms;
  h.n_rns = db->n_rns;
  h.n_p2 = db->n_p2;
  h.n_primes = db->keys->n_primes;
  expected_bytes(db, h.bytes);
  const DevBuf* bufs[4] = {&db->Dt, &db->digits, &db->rns, &db->p2};
  for (int i = 0; i < 4; ++i)
    if (h.bytes[i] && (!bufs[i]->ptr || bufs[i]->bytes < h.bytes[i]))
      return fail(HFE_EINTERNAL, "database buffer smaller than its layout");
  File f;
  f.f = std::fopen(path, "wb");
  if (!f.f) return fail(HFE_EINVAL, std::string("cannot open for writing: ") + path);
  if (std::fwrite(&h, sizeof(h), 1, f.f) != 1) return fail(HFE_EINVAL, "write failed");
  Pinned stage;
  HFE_CHECK_HIP(hipHostMalloc(&stage.p, kStage, hipHostMallocDefault));
  for (int i = 0; i < 4; ++i) {
    const uint8_t* src = bufs[i]->as<uint8_t>();
    for (uint64_t off = 0; off < h.bytes[i]; off += kStage) {
      const size_t n = (size_t)std::min<uint64_t>(kStage, h.bytes[i] - off);
      HFE_CHECK_HIP(hipMemcpyAsync(stage.p, src + off, n, hipMemcpyDeviceToHost, s));
      HFE_CHECK_HIP(hipStreamSynchronize(s));
      if (std::fwrite(stage.p, 1, n, f.f) != n) return fail(HFE_EINVAL, "write failed");
    }
  }
  if (std::fclose(f.f) != 0) {
    f.f = nullptr;
    return fail(HFE_EINVAL, "write failed");
  }
  f.f = nullptr;
  return HFE_OK;
}

hfe_status hfe_db_bytes(const hfe_db* db, uint32_t form, size_t* bytes) {
  const HandleBase* hb = static_cast<const HandleBase*>(static_cast<const void*>(db));
  if (!db || hb->kind != kDb || !bytes) return fail(HFE_EINVAL, "invalid database handle or bytes");
  if (form != 0 && form != HFE_FORM_PLAIN_U64 && form != HFE_FORM_I8_MFMA && form != HFE_FORM_RNS_I8 &&
      form != HFE_FORM_P2_I8)
    return fail(HFE_EINVAL, "form must be 0 or one hfe_form");
  if (form != 0 && !(db->forms & form)) return fail(HFE_EINVAL, "database not prepared for this form");
  uint64_t b[4];
  expected_bytes(db, b);
  const uint32_t form_of[4] = {HFE_FORM_PLAIN_U64, HFE_FORM_I8_MFMA, HFE_FORM_RNS_I8, HFE_FORM_P2_I8};
  size_t total = 0;
  for (int i = 0; i < 4; ++i)
    if (form == 0 || form == form_of[i]) total += (size_t)b[i];
  *bytes = total;
  return HFE_OK;
}

hfe_status hfe_db_load(const hfe_keys* keys, const char* path, uint32_t forms, void* stream, hfe_db** out) {
  if (!out) return fail(HFE_EINVAL, "out is NULL");
  *out = nullptr;
  const HandleBase* hb = static_cast<const HandleBase*>(static_cast<const void*>(keys));
  if (!keys || hb->kind != kKeys) return fail(HFE_EINVAL, "invalid keys handle");
  if (!path) return fail(HFE_EINVAL, "path is NULL");
  if (keys->family != 0) return fail(HFE_EINVAL, "databases of the n^2 modulus chain are not stored");
  const hipStream_t s = (hipStream_t)stream;
  File f;
  f.f = std::fopen(path, "rb");
  if (!f.f) return fail(HFE_EINVAL, std::string("cannot open for reading: ") + path);
  FileHeader h;
  if (std::fread(&h, sizeof(h), 1, f.f) != 1 || std::memcmp(h.magic, kMagic, sizeof(kMagic)) != 0)
    return fail(HFE_EINVAL, "not a database file of this library version");
  if (h.key_print != key_print(keys)) return fail(HFE_EINVAL, "the database was written under other keys");
  const hfe_params& P = keys->P;
  const int64_t ndb = 1ll << P.log_n_db, nq = 1ll << P.log_n_q;
  if (h.d1 < 1 || h.d1 > (int64_t)P.max_db_rows || h.R != ndb + h.d1 || h.K != (int64_t)P.d2 + nq ||
      h.KB != (h.K + kKB - 1) / kKB || h.R_pad != (h.R + 63) / 64 * 64 + kRowPad || h.n_primes != keys->n_primes ||
      h.forms == 0 || (h.forms & ~15u) || h.n_rns < 0 || h.n_rns > kRnsMaxMods || h.n_p2 < 0 ||
      h.n_p2 > kP2MaxBases || ((h.forms & HFE_FORM_RNS_I8) && h.n_rns < 1) ||
      ((h.forms & HFE_FORM_P2_I8) && h.n_p2 < 1))
    return fail(HFE_EINVAL, "database file header does not match the keys");
  if (forms == 0) forms = h.forms;
  if ((forms & ~h.forms) != 0) return fail(HFE_EINVAL, "the file does not hold every requested form");
  std::unique_ptr<hfe_db> D(new (std::nothrow) hfe_db());
  if (!D) return fail(HFE_ENOMEM, "host allocation failed");
  D->kind = kDb;
  D->stream = s;
  D->keys = keys;
  D->d1 = h.d1;
  D->R = h.R;
  D->K = h.K;
  D->KB = h.KB;
  D->R_pad = h.R_pad;
  D->forms = h.forms;
  D->n_rns = (h.forms & HFE_FORM_RNS_I8) ? h.n_rns : 0;
  D->n_p2 = (h.forms & HFE_FORM_P2_I8) ? h.n_p2 : 0;
  D->slots_plain = D->slots_planes = keys->n_primes;
  uint64_t want[4];
  expected_bytes(D.get(), want);
  for (int i = 0; i < 4; ++i)
    if (want[i] != h.bytes[i]) return fail(HFE_EINVAL, "database file sizes do not match its header");
  // the requested forms only; the others' bytes are skipped in the file
  D->forms = forms;
  const uint32_t form_of[4] = {HFE_FORM_PLAIN_U64, HFE_FORM_I8_MFMA, HFE_FORM_RNS_I8, HFE_FORM_P2_I8};
  if (!(forms & HFE_FORM_RNS_I8)) D->n_rns = 0;
  if (!(forms & HFE_FORM_P2_I8)) D->n_p2 = 0;
  DevBuf* bufs[4] = {&D->Dt, &D->digits, &D->rns, &D->p2};
  Pinned stage;
  HFE_CHECK_HIP(hipHostMalloc(&stage.p, kStage, hipHostMallocDefault));
  for (int i = 0; i < 4; ++i) {
    if (!h.bytes[i]) continue;
    if (!(forms & form_of[i])) {
      if (std::fseek(f.f, (long)h.bytes[i], SEEK_CUR) != 0) return fail(HFE_EINVAL, "database file is truncated");
      continue;
    }
    HFE_TRY(bufs[i]->alloc((size_t)h.bytes[i], s));
    uint8_t* dst = bufs[i]->as<uint8_t>();
    for (uint64_t off = 0; off < h.bytes[i]; off += kStage) {
      const size_t n = (size_t)std::min<uint64_t>(kStage, h.bytes[i] - off);
      // the previous chunk's copy has finished reading the staging buffer
      HFE_CHECK_HIP(hipStreamSynchronize(s));
      if (std::fread(stage.p, 1, n, f.f) != n) {
        HFE_CHECK_HIP(hipStreamSynchronize(s));
        return fail(HFE_EINVAL, "database file is truncated");
      }
      HFE_CHECK_HIP(hipMemcpyAsync(dst + off, stage.p, n, hipMemcpyHostToDevice, s));
    }
  }
  HFE_CHECK_HIP(hipStreamSynchronize(s));
  char extra;
  if (std::fread(&extra, 1, 1, f.f) != 0) return fail(HFE_EINVAL, "database file has trailing bytes");
  *out = D.release();
  return HFE_OK;
}

}  // extern "C"
