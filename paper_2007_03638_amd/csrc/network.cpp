// Contraction-program planner and executor (see network.h).
#include "network.h"

#include "vec.h"

#include <algorithm>
#include <cctype>
#include <sstream>

namespace mera {

namespace {

std::string trim(const std::string& s) {
  size_t a = s.find_first_not_of(" \t"), b = s.find_last_not_of(" \t");
  return a == std::string::npos ? std::string() : s.substr(a, b - a + 1);
}

// "NAME[labels]" -> (NAME, labels)
std::pair<std::string, std::string> parse_ref(const std::string& tok) {
  std::string t = trim(tok);
  size_t lb = t.find('['), rb = t.find(']');
  if (lb == std::string::npos || rb == std::string::npos || rb < lb)
    throw Error(MERA_EINVAL, "bad tensor reference '" + t + "'");
  return {trim(t.substr(0, lb)), t.substr(lb + 1, rb - lb - 1)};
}

int64_t roundup(int64_t x, int64_t m) { return ((x + m - 1) / m) * m; }

}  // namespace

int Program::id(const std::string& n) const {
  for (size_t i = 0; i < tensors.size(); ++i)
    if (tensors[i] == n) return (int)i;
  return -1;
}

Program Program::parse(const std::string& name, const std::vector<std::string>& lines,
                       const std::vector<std::string>& externals) {
  Program p;
  p.name = name;
  auto get = [&](const std::string& n, const std::string& labels) {
    int i = p.id(n);
    if (i < 0) {
      p.tensors.push_back(n);
      p.layout.push_back(labels);
      p.external.push_back(std::find(externals.begin(), externals.end(), n) != externals.end());
      return (int)p.tensors.size() - 1;
    }
    if (p.layout[i].size() != labels.size())
      throw Error(MERA_EINVAL, "rank mismatch for tensor " + n + " in program " + name);
    return i;
  };
  std::vector<std::string> zero_names;
  for (const std::string& raw : lines) {
    std::string line = trim(raw);
    if (line.empty()) continue;
    if (line.rfind("@loop", 0) == 0) {
      std::string leg = trim(line.substr(5));
      if (leg.size() != 1 || p.loop_begin >= 0) throw Error(MERA_EINVAL, "bad @loop in program " + name);
      p.slice_leg = leg[0];
      p.loop_begin = (int)p.steps.size();
      continue;
    }
    if (line == "@end") {
      if (p.loop_begin < 0 || p.loop_end >= 0) throw Error(MERA_EINVAL, "bad @end in program " + name);
      p.loop_end = (int)p.steps.size();
      continue;
    }
    if (line.rfind("@zero", 0) == 0) {
      std::stringstream zs(line.substr(5));
      std::string t;
      while (zs >> t) zero_names.push_back(t);
      continue;
    }
    bool acc = false;
    size_t eq = line.find("+=");
    if (eq != std::string::npos) {
      acc = true;
    } else {
      eq = line.find('=');
      if (eq == std::string::npos) throw Error(MERA_EINVAL, "no '=' in '" + line + "'");
    }
    std::string lhs = line.substr(0, eq);
    std::string rhs = line.substr(eq + (acc ? 2 : 1));
    std::vector<std::string> parts;
    std::stringstream ss(rhs);
    std::string tok;
    while (std::getline(ss, tok, '*')) parts.push_back(trim(tok));
    double alpha = 1.0;
    if (parts.size() == 3) {
      alpha = std::stod(parts[0]);
      parts.erase(parts.begin());
    }
    if (parts.size() != 2) throw Error(MERA_EINVAL, "need two operands in '" + line + "'");
    auto c = parse_ref(lhs), a = parse_ref(parts[0]), b = parse_ref(parts[1]);
    StepDef st;
    st.a = get(a.first, a.second);
    st.b = get(b.first, b.second);
    st.c = get(c.first, c.second);
    st.la = a.second;
    st.lb = b.second;
    st.lc = c.second;
    st.alpha = alpha;
    st.accumulate = acc;
    p.steps.push_back(st);
  }
  if (p.loop_begin >= 0 && p.loop_end < 0) throw Error(MERA_EINVAL, "unterminated @loop in program " + name);
  p.produced_at.assign(p.tensors.size(), -1);
  for (size_t si = 0; si < p.steps.size(); ++si)
    if (p.produced_at[p.steps[si].c] < 0 && !p.external[p.steps[si].c]) p.produced_at[p.steps[si].c] = (int)si;
  for (const std::string& z : zero_names) {
    int i = p.id(z);
    if (i < 0 || p.external[i]) throw Error(MERA_EINVAL, "bad @zero tensor " + z + " in program " + name);
    p.zero_before.push_back(i);
  }
  return p;
}

namespace {

// Row-major strides of a tensor whose axes carry labels `lab` with extents from `dims`.
std::vector<int64_t> strides_of(const std::string& lab, const LegDims& dims) {
  std::vector<int64_t> s(lab.size());
  int64_t acc = 1;
  for (int i = (int)lab.size() - 1; i >= 0; --i) {
    s[i] = acc;
    acc *= dims[(unsigned char)lab[i]];
  }
  return s;
}

int64_t stride_of(const std::string& lab, const std::vector<int64_t>& st, char c) {
  size_t pos = lab.find(c);
  return pos == std::string::npos ? 0 : st[pos];
}

// Offsets of the flattened index over `legs` (last fastest) for a tensor with labels/strides.
void fill_table(std::vector<int64_t>& out, const std::string& legs, const LegDims& dims, const std::string& lab,
                const std::vector<int64_t>& st, int64_t padded) {
  int64_t total = 1;
  for (char c : legs) total *= dims[(unsigned char)c];
  out.assign(padded, 0);
  std::vector<int64_t> idx(legs.size(), 0), sl(legs.size());
  for (size_t i = 0; i < legs.size(); ++i) sl[i] = stride_of(lab, st, legs[i]);
  int64_t off = 0;
  for (int64_t f = 0; f < total; ++f) {
    out[f] = off;
    // increment multi-index (last fastest), maintain offset
    for (int i = (int)legs.size() - 1; i >= 0; --i) {
      idx[i]++;
      off += sl[i];
      if (idx[i] < dims[(unsigned char)legs[i]]) break;
      off -= sl[i] * idx[i];
      idx[i] = 0;
    }
  }
}

// Contracted legs as a mixed-radix k index for the kernels, fastest first (the last leg of `Kl` is the fastest):
// legs of extent 1 are dropped, and a leg that continues the previous one contiguously in both operands is merged
// into it. Each leg's reciprocal multiplier is checked exact for every quotient the kernels will form; the slowest
// leg gets none (its digit is the remaining quotient).
GettKLegs k_legs(const std::string& prog, const std::string& Kl, const LegDims& dims, const std::string& LA,
                 const std::vector<int64_t>& sa, const std::string& LB, const std::vector<int64_t>& sb, int64_t K) {
  struct Leg {
    int64_t ext, xa, xb;
  };
  std::vector<Leg> legs;
  for (int i = (int)Kl.size() - 1; i >= 0; --i) {
    const char c = Kl[i];
    const int64_t e = dims[(unsigned char)c];
    if (e == 1) continue;
    const int64_t xa = stride_of(LA, sa, c), xb = stride_of(LB, sb, c);
    if (!legs.empty() && legs.back().xa * legs.back().ext == xa && legs.back().xb * legs.back().ext == xb)
      legs.back().ext *= e;
    else
      legs.push_back(Leg{e, xa, xb});
  }
  if ((int)legs.size() > kGettMaxKLegs)
    throw Error(MERA_EINVAL, prog + ": more than " + std::to_string(kGettMaxKLegs) + " contracted legs");
  if (K >= (int64_t(1) << 31)) throw Error(MERA_EINVAL, prog + ": contracted extent too large");
  GettKLegs kl;
  kl.n = (int)legs.size();
  for (const Leg& l : legs)
    if (l.xa < 0 || l.xb < 0 || l.xa >= (int64_t(1) << 32) || l.xb >= (int64_t(1) << 32))
      throw Error(MERA_EINVAL, prog + ": contracted-leg stride outside 32 bits");
  int64_t below = 1;  // product of the faster extents
  for (int l = 0; l < kl.n; ++l) {
    const uint64_t e = (uint64_t)legs[l].ext;
    kl.ext[l] = (uint32_t)e;
    if (l + 1 < kl.n) {
      const uint64_t qmax = (uint64_t)(K - 1) / (uint64_t)below;  // largest quotient entering leg l
      if (qmax * e > (uint64_t(1) << 32)) throw Error(MERA_EINVAL, prog + ": contracted leg too large");
      kl.mag[l] = (uint32_t)(((uint64_t(1) << 32) + e - 1) / e);
    }  // the slowest leg takes the whole remaining quotient: mag 0 (no division)
    kl.sa[l] = (uint32_t)legs[l].xa;
    kl.sb[l] = (uint32_t)legs[l].xb;
    below *= (int64_t)e;
  }
  return kl;
}

// The kernels' k offset (digit extraction by reciprocal multiplication over NKL legs in 32-bit arithmetic,
// digit-stride products accumulated in 64 bits), on the host.
int64_t host_k_offset(uint32_t k, const GettKLegs& kl, const uint32_t* stride, int nkl) {
  uint64_t off = 0;
  uint32_t q = k;
  for (int l = 0; l + 1 < nkl; ++l) {
    const uint32_t qn = (uint32_t)(((uint64_t)q * kl.mag[l]) >> 32);
    off += (uint64_t)(q - qn * kl.ext[l]) * stride[l];
    q = qn;
  }
  return (int64_t)(off + (uint64_t)q * stride[nkl - 1]);
}

// Checks the arithmetic k offsets against the explicit offset tables of A and B, once per planned step.
void check_k_legs(const std::string& prog, const GettKLegs& kl, const std::string& Kl, const LegDims& dims,
                  const std::string& LA, const std::vector<int64_t>& sa, const std::string& LB,
                  const std::vector<int64_t>& sb, int64_t K) {
  std::vector<int64_t> ta, tb;
  fill_table(ta, Kl, dims, LA, sa, K);
  fill_table(tb, Kl, dims, LB, sb, K);
  const int nkl = kl.n <= 2 ? 2 : kGettMaxKLegs;
  for (int64_t k = 0; k < K; ++k)
    if (host_k_offset((uint32_t)k, kl, kl.sa, nkl) != ta[k] || host_k_offset((uint32_t)k, kl, kl.sb, nkl) != tb[k])
      throw Error(MERA_EINVAL, prog + ": contracted-leg offsets disagree with the leg strides");
}

// `dims` gives the index ranges of the step; sdims[0..2] give the extents used for the storage strides of A, B
// and C (they differ from `dims` only in the loop leg of a full-extent tensor addressed chunk by chunk).
PlanCache::Entry& plan_step(Ctx& ctx, const Program& prog, size_t si, const LegDims& dims,
                            const LegDims* const sdims[3]) {
  const StepDef& s = prog.steps[si];
  std::string key = prog.name + "#" + std::to_string(si);
  std::string all = s.la + s.lb + s.lc;
  std::sort(all.begin(), all.end());
  all.erase(std::unique(all.begin(), all.end()), all.end());
  for (char c : all) key += ":" + std::to_string(dims[(unsigned char)c]);
  if (prog.slice_leg) {
    const unsigned char L = (unsigned char)prog.slice_leg;
    for (int o = 0; o < 3; ++o) key += "/" + std::to_string((*sdims[o])[L]);
  }
  std::lock_guard<std::mutex> lock(ctx.plans->mu);
  auto it = ctx.plans->map.find(key);
  if (it != ctx.plans->map.end()) return *it->second;

  auto has = [](const std::string& s_, char c) { return s_.find(c) != std::string::npos; };
  // The kernels' lanes run along N when they store C. When C's unit-stride leg comes from A (an M leg), the
  // roles of A and B are exchanged (C^T = B^T A^T) so that the stores stay coalesced.
  const bool swap = has(s.la, s.lc.back());
  const std::string& LA = swap ? s.lb : s.la;
  const std::string& LB = swap ? s.la : s.lb;
  const LegDims& DA = swap ? *sdims[1] : *sdims[0];
  const LegDims& DB = swap ? *sdims[0] : *sdims[1];
  std::string Ml, Nl, Kl;
  for (char c : LA) {
    bool inb = has(LB, c), inc = has(s.lc, c);
    if (inc && !inb) Ml += c;
    else if (inb && !inc) Kl += c;
    else throw Error(MERA_EINVAL, prog.name + ": leg '" + std::string(1, c) + "' of A is batch or traced");
  }
  for (char c : LB) {
    bool ina = has(LA, c), inc = has(s.lc, c);
    if (inc && !ina) Nl += c;
    else if (!(ina && !inc)) throw Error(MERA_EINVAL, prog.name + ": leg of B is batch or traced");
  }
  for (char c : s.lc)
    if (!has(Ml, c) && !has(Nl, c)) throw Error(MERA_EINVAL, prog.name + ": output leg not produced");
  if (Ml.size() + Nl.size() != s.lc.size()) throw Error(MERA_EINVAL, prog.name + ": repeated output leg");
  for (char c : all)
    if (dims[(unsigned char)c] <= 0) throw Error(MERA_EINVAL, prog.name + ": unset leg extent");

  const bool a_kfast = !Kl.empty() && has(Kl, LA.back());
  const bool b_kfast = !Kl.empty() && has(Kl, LB.back());
  if (!a_kfast && b_kfast) {
    // order K legs as B stores them so B's unit-stride leg is fastest in k
    std::string k2;
    for (char c : LB)
      if (has(Kl, c)) k2 += c;
    Kl = k2;
  }
  auto ext = [&](const std::string& legs) {
    int64_t t = 1;
    for (char c : legs) t *= dims[(unsigned char)c];
    return t;
  };
  const int64_t M = ext(Ml), N = ext(Nl), K = ext(Kl);
  const int64_t Mp = roundup(M, 128), Np = roundup(N, 128);
  auto sa = strides_of(LA, DA), sb = strides_of(LB, DB), sc = strides_of(s.lc, *sdims[2]);
  const GettKLegs kl = k_legs(prog.name, Kl, dims, LA, sa, LB, sb, K);
  check_k_legs(prog.name, kl, Kl, dims, LA, sa, LB, sb, K);
  std::vector<int64_t> host;
  host.reserve(2 * Mp + 2 * Np);
  std::vector<int64_t> tmp;
  size_t off_am, off_bn, off_cm, off_cn;
  off_am = host.size(); fill_table(tmp, Ml, dims, LA, sa, Mp); host.insert(host.end(), tmp.begin(), tmp.end());
  off_bn = host.size(); fill_table(tmp, Nl, dims, LB, sb, Np); host.insert(host.end(), tmp.begin(), tmp.end());
  off_cm = host.size(); fill_table(tmp, Ml, dims, s.lc, sc, Mp); host.insert(host.end(), tmp.begin(), tmp.end());
  off_cn = host.size(); fill_table(tmp, Nl, dims, s.lc, sc, Np); host.insert(host.end(), tmp.begin(), tmp.end());

  auto e = std::make_unique<PlanCache::Entry>();
  e->tables.alloc(host.size() * sizeof(int64_t));
  // stream-ordered upload (the host vector lives until the sync); no work on the legacy null stream
  MERA_HIP(hipMemcpyAsync(e->tables.ptr, host.data(), host.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                          ctx.stream));
  MERA_HIP(hipStreamSynchronize(ctx.stream));
  const int64_t* base = e->tables.as<int64_t>();
  e->t.a_m = base + off_am;
  e->t.b_n = base + off_bn;
  e->t.c_m = base + off_cm;
  e->t.c_n = base + off_cn;
  e->t.kl = kl;
  e->t.M = M;
  e->t.N = N;
  e->t.K = K;
  e->t.a_kfast = a_kfast;
  e->t.b_kfast = b_kfast;
  // vector width of the tile loads each operand's layout allows
  auto vec_width = [&](const std::string& L, const std::vector<int64_t>& st, const std::string& walk) {
    if (walk.empty() || walk.back() != L.back()) return 1;
    for (int w : {4, 2}) {
      bool ok = dims[(unsigned char)L.back()] % w == 0;
      for (size_t i = 0; i + 1 < L.size(); ++i) ok = ok && st[i] % w == 0;
      if (ok) return w;
    }
    return 1;
  };
  e->t.a_vw = vec_width(LA, sa, a_kfast ? Kl : Ml);
  e->t.b_vw = vec_width(LB, sb, b_kfast ? Kl : Nl);
  e->macs = (double)M * (double)N * (double)K;
  e->swap = swap;
  auto& ref = *e;
  ctx.plans->map.emplace(key, std::move(e));
  return ref;
}

}  // namespace

double run_group(Ctx& lead, const Program& prog, const LegDims& dims, const std::vector<Binding>& group, Prec prec,
                 int64_t chunk, bool prepare_only, std::vector<const void*>* touched) {
  const int G = (int)group.size();
  if (G < 1 || G > kGettMaxGroup) throw Error(MERA_EINVAL, prog.name + ": group size out of range");
  for (const Binding& b : group)
    if (!b.ctx || b.ext.size() != prog.tensors.size()) throw Error(MERA_EINVAL, prog.name + ": binding count");
  const size_t eb = elem_bytes(prec);
  const unsigned char L = (unsigned char)prog.slice_leg;
  const bool sliced = prog.slice_leg && chunk > 0 && chunk < dims[L];
  if (sliced && dims[L] % chunk != 0) throw Error(MERA_EINVAL, prog.name + ": chunk must divide the loop leg");
  LegDims cdims = dims;
  if (sliced) cdims[L] = chunk;
  auto in_loop = [&](int si) { return sliced && si >= prog.loop_begin && si < prog.loop_end; };
  // a tensor is "inner" when the loop creates it; inner tensors are allocated with one chunk of the leg
  auto inner = [&](int t) {
    return sliced && prog.produced_at[t] >= prog.loop_begin && prog.produced_at[t] < prog.loop_end;
  };
  const size_t nt = prog.tensors.size();
  std::vector<void*> ptr(nt * G, nullptr);  // ptr[g * nt + i]
  for (int g = 0; g < G; ++g)
    for (size_t i = 0; i < nt; ++i) {
      void*& p = ptr[g * nt + i];
      if (prog.external[i]) {
        if (!group[g].ext[i]) throw Error(MERA_EINVAL, prog.name + ": unbound tensor " + prog.tensors[i]);
        p = group[g].ext[i];
      } else {
        const LegDims& d = inner((int)i) ? cdims : dims;
        int64_t n = 1;
        for (char c : prog.layout[i]) n *= d[(unsigned char)c];
        p = group[g].ctx->buf("net/" + prog.tensors[i], (size_t)n * eb);
      }
    }
  double macs = 0;  // per binding
  auto launch = [&](size_t si, const LegDims& idims, int64_t c0) {
    const StepDef& s = prog.steps[si];
    const int ids[3] = {s.a, s.b, s.c};
    const std::string* labs[3] = {&s.la, &s.lb, &s.lc};
    const LegDims* sd[3];
    size_t shift[3];
    for (int o = 0; o < 3; ++o) {
      const bool full = !in_loop((int)si) || !inner(ids[o]);
      sd[o] = full ? &dims : &cdims;
      shift[o] = 0;
      const size_t pos = labs[o]->find((char)L);
      if (in_loop((int)si) && full && pos != std::string::npos) {
        // full-extent tensor addressed at this chunk of the loop leg
        int64_t stride = 1;
        for (size_t j = pos + 1; j < labs[o]->size(); ++j) stride *= dims[(unsigned char)(*labs[o])[j]];
        shift[o] = (size_t)(c0 * stride) * eb;
      }
    }
    PlanCache::Entry& e = plan_step(lead, prog, si, idims, sd);
    GettLaunch l;
    l.groups = G;
    const int oa = e.swap ? 1 : 0, ob = 1 - oa;  // operand roles (exchanged for an m-fast C)
    for (int g = 0; g < G; ++g) {
      l.A[g] = static_cast<char*>(ptr[g * nt + ids[oa]]) + shift[oa];
      l.B[g] = static_cast<char*>(ptr[g * nt + ids[ob]]) + shift[ob];
      l.C[g] = static_cast<char*>(ptr[g * nt + ids[2]]) + shift[2];
    }
    l.alpha = s.alpha;
    l.beta = s.accumulate ? 1.0 : 0.0;
    l.prec = prec;
    l.splits = 0;
    l.prepare_only = prepare_only;
    gett_run(lead, e.t, l);
    macs += e.macs;
  };
  const int lb = prog.loop_begin >= 0 ? prog.loop_begin : 0;
  const int le = prog.loop_end >= 0 ? prog.loop_end : 0;
  for (int si = 0; si < lb; ++si) launch(si, dims, 0);
  if (!prepare_only)
    for (int t : prog.zero_before) {
      int64_t n = 1;
      for (char c : prog.layout[t]) n *= dims[(unsigned char)c];
      for (int g = 0; g < G; ++g) fill(lead, VPtr{ptr[g * nt + t], prec}, n, 0.0);
    }
  if (sliced) {
    for (int64_t c0 = 0; c0 < dims[L]; c0 += chunk)
      for (int si = lb; si < le; ++si) launch(si, cdims, c0);
  } else {
    for (int si = lb; si < le; ++si) launch(si, dims, 0);
  }
  for (size_t si = le; si < prog.steps.size(); ++si) launch(si, dims, 0);
  if (touched) {
    touched->assign(ptr.begin(), ptr.end());
    auto it = lead.scratch.find("gett.partial");
    touched->push_back(it == lead.scratch.end() ? nullptr : it->second.ptr);
  }
  if (!prepare_only)
    for (int g = 0; g < G; ++g) group[g].ctx->macs += macs;
  return macs;
}

void run_program(Ctx& ctx, const Program& prog, const LegDims& dims, const std::vector<void*>& ext, Prec prec,
                 int64_t chunk) {
  if (ext.size() != prog.tensors.size()) throw Error(MERA_EINVAL, prog.name + ": binding count");
  if (ctx.batcher) {
    ctx.batcher->run(ctx, prog, dims, ext, prec, chunk);
    return;
  }
  run_group(ctx, prog, dims, {Binding{&ctx, ext}}, prec, chunk, false, nullptr);
}

void run_program(Ctx& ctx, const Program& prog, const LegDims& dims,
                 const std::vector<std::pair<std::string, void*>>& bind, Prec prec, int64_t chunk) {
  std::vector<void*> ext(prog.tensors.size(), nullptr);
  for (auto& b : bind) {
    int i = prog.id(b.first);
    if (i < 0) continue;
    ext[i] = b.second;
  }
  run_program(ctx, prog, dims, ext, prec, chunk);
}

}  // namespace mera
