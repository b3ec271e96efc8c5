"""Seeded synthetic genomes and reads shaped like the paper's workloads.

This module is shared by the tests, the benchmark and the smoke check, and it feeds both
the GPU library and the CPU oracle.  It holds none of the method's arithmetic: it draws
bases, copies segments, introduces sequencing errors and reverse-complements reads the
way a sequencer would, and nothing else (no sparsification, k-mers, hashing, minimizers,
sorting or lookups).

Sequences are returned as one base code per byte (A=0, C=1, G=2, T=3) plus int64
offsets[n_seq+1].  Every generator takes an explicit seed and draws from
numpy.random.default_rng (PCG64) in a fixed order, so the same call always returns the
same bytes.

Shapes follow the paper's workloads (Results; Supplementary Table 1):
  * Illumina-like reads: 150 bp, both strands, substitutions (+ rare 1-bp indels);
  * HiFi-like reads: length ~ Normal(15 kb, 3 kb), 1 % errors (sub/ins/del 50/25/25);
  * ONT-like reads: lognormal length with mean 10 kb and sigma 1.51 (the paper's ONT
    mean/median ratio), 8 % errors (50/25/25); all long reads clamped to
    [1 kb, 1,331,423 bp] (the paper's 1 kb filter and longest ONT read);
  * references: i.i.d. uniform bases plus 5 % repeat content made of 5 kb segments
    copied 10 times at 2 % divergence in random orientation.
"""
import numpy as np

LONG_MIN = 1000
LONG_MAX = 1331423


def revcomp(codes):
    """Reverse complement of a code array (the opposite DNA strand; N stays N)."""
    r = np.asarray(codes, np.uint8)[::-1]
    return np.where(r == 4, 4, 3 - r).astype(np.uint8)


def random_genome(length, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 4, size=int(length), dtype=np.uint8)


def _substitute(rng, seq, rate):
    mask = rng.random(seq.shape) < rate
    nsub = int(mask.sum())
    if nsub:
        seq[mask] = (seq[mask] + rng.integers(1, 4, size=nsub, dtype=np.uint8)) % 4
    return seq


def add_repeats(genome, seed, frac=0.05, seg_len=5000, copies=10, divergence=0.02):
    """Overwrite frac of the genome with repeat families: each family is a random
    seg_len consensus written `copies` times, each copy with `divergence` i.i.d.
    substitutions and a random orientation, at distinct non-overlapping slots."""
    g = genome.copy()
    rng = np.random.default_rng(seed)
    L = g.size
    families = int(round(frac * L / (seg_len * copies)))
    n_slots = L // seg_len
    if families == 0 or n_slots < families * copies:
        return g
    slots = rng.choice(n_slots, size=families * copies, replace=False)
    for f in range(families):
        cons = rng.integers(0, 4, size=seg_len, dtype=np.uint8)
        for c in range(copies):
            cp = _substitute(rng, cons.copy(), divergence)
            if rng.integers(0, 2):
                cp = revcomp(cp)
            pos = int(slots[f * copies + c]) * seg_len
            g[pos:pos + seg_len] = cp
    return g


def fixed_reads(ref, n, length, seed, sub=0.01, ins=0.0, dele=0.0, margin=16):
    """n reads of exactly `length` bases sampled uniformly from both strands of ref.

    Returns (codes, offsets, start, strand) where start is the 0-based reference start
    of the sampled template and strand 1 means the read is the reverse complement."""
    rng = np.random.default_rng(seed)
    L = ref.size
    span = length + margin
    if L < span:
        raise ValueError("reference shorter than a read")
    starts = rng.integers(0, L - span + 1, size=n)
    strands = rng.integers(0, 2, size=n).astype(np.uint8)
    idx = starts[:, None] + np.arange(span)[None, :]
    seg = ref[idx]
    _substitute(rng, seg, sub)
    reads = seg[:, :length].copy()
    if ins > 0 or dele > 0:
        ev = rng.random((n, span)) < (ins + dele)
        rows = np.nonzero(ev[:, :length].any(axis=1))[0]
        for r in rows:
            # a row with an indel event is redrawn from its template with the full
            # sequential sub/ins/del model, then trimmed (or padded) to `length`
            tpl = ref[starts[r]:starts[r] + span]
            m = _mutate_indel_fast(rng, tpl, sub, ins, dele)[:length]
            if m.size < length:
                m = np.concatenate([m, rng.integers(0, 4, size=length - m.size, dtype=np.uint8)])
            reads[r] = m
    rev = strands == 1
    flipped = reads[rev][:, ::-1]
    reads[rev] = np.where(flipped == 4, 4, 3 - flipped)
    offsets = np.arange(0, (n + 1) * length, length, dtype=np.int64)
    return reads.reshape(-1).copy(), offsets, starts.astype(np.int64), strands


def variable_reads(ref, lengths, seed, sub, ins, dele):
    """One read per entry of `lengths`, sampled from both strands with the sequential
    sub/ins/del model.  Returns (codes, offsets, start, strand)."""
    rng = np.random.default_rng(seed)
    L = ref.size
    parts, starts, strands = [], [], []
    for ln in lengths:
        ln = int(min(ln, L))
        st = int(rng.integers(0, L - ln + 1))
        s = int(rng.integers(0, 2))
        tpl = ref[st:st + ln]
        r = _mutate_indel_fast(rng, tpl, sub, ins, dele)
        if s:
            r = revcomp(r)
        parts.append(r)
        starts.append(st)
        strands.append(s)
    offsets = np.zeros(len(parts) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([p.size for p in parts])
    codes = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
    return codes, offsets, np.array(starts, np.int64), np.array(strands, np.uint8)


def _mutate_indel_fast(rng, tpl, sub, ins, dele):
    """Vectorised form of the sequential sub/ins/del model (no trimming)."""
    n = tpl.size
    u = rng.random(n)
    keep = u >= dele
    subm = (u >= dele) & (u < dele + sub)
    base = tpl.copy()
    ns = int(subm.sum())
    if ns:
        base[subm] = (base[subm] + rng.integers(1, 4, size=ns, dtype=np.uint8)) % 4
    insm = rng.random(n) < ins
    ni = int(insm.sum())
    ins_b = rng.integers(0, 4, size=ni, dtype=np.uint8)
    # each template position contributes [base if kept] + [inserted base if insm]
    cnt = keep.astype(np.int64) + insm.astype(np.int64)
    out = np.empty(int(cnt.sum()), dtype=np.uint8)
    pos = np.cumsum(cnt) - cnt
    out[pos[keep]] = base[keep]
    out[(pos + keep.astype(np.int64))[insm]] = ins_b
    return out


def hifi_lengths(n, rng):
    ln = rng.normal(15000.0, 3000.0, size=n)
    return np.clip(np.round(ln), LONG_MIN, LONG_MAX).astype(np.int64)


def ont_lengths(n, rng, mean=10000.0, sigma=1.51):
    mu = np.log(mean) - sigma * sigma / 2.0
    ln = rng.lognormal(mu, sigma, size=n)
    return np.clip(np.round(ln), LONG_MIN, LONG_MAX).astype(np.int64)


def concat(batches):
    """Concatenate (codes, offsets, ...) batches into one batch."""
    codes = np.concatenate([b[0] for b in batches])
    offs = [np.asarray(batches[0][1], np.int64)]
    base = offs[0][-1]
    for b in batches[1:]:
        o = np.asarray(b[1], np.int64)
        offs.append(o[1:] + base)
        base += o[-1]
    return codes, np.concatenate(offs)


def genome_db(n_genomes, seed, min_len=1_000_000, max_len=5_000_000, shared_frac=0.3,
              block_frac=0.10, divergence=0.05):
    """Containment database: n_genomes i.i.d. genomes with uniform lengths; a fraction
    `shared_frac` of them receives one contiguous block of block_frac of its length copied
    from one random partner with `divergence` substitutions."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(min_len, max_len + 1, size=n_genomes)
    genomes = [rng.integers(0, 4, size=int(l), dtype=np.uint8) for l in lens]
    rs = np.random.default_rng(seed + 200)
    n_shared = int(round(shared_frac * n_genomes))
    receivers = rs.choice(n_genomes, size=n_shared, replace=False)
    for g in receivers:
        partner = int(rs.integers(0, n_genomes - 1))
        if partner >= g:
            partner += 1
        blen = int(block_frac * genomes[g].size)
        blen = min(blen, genomes[partner].size)
        src = int(rs.integers(0, genomes[partner].size - blen + 1))
        dst = int(rs.integers(0, genomes[g].size - blen + 1))
        genomes[g][dst:dst + blen] = _substitute(rs, genomes[partner][src:src + blen].copy(),
                                                 divergence)
    offsets = np.zeros(n_genomes + 1, np.int64)
    offsets[1:] = np.cumsum(lens)
    return np.concatenate(genomes), offsets


def sample_from_genomes(codes, offsets, n_reads, n_source, length, seed, sub=0.01):
    """n_reads reads of `length` bases from n_source randomly chosen genomes with
    lognormal(0, 1) abundances (normalised), both strands, i.i.d. substitutions.
    Returns (read codes, read offsets, source genome of each read)."""
    rng = np.random.default_rng(seed)
    n_gen = offsets.size - 1
    src = rng.choice(n_gen, size=n_source, replace=False)
    ab = rng.lognormal(0.0, 1.0, size=n_source)
    ab /= ab.sum()
    which = src[rng.choice(n_source, size=n_reads, p=ab)]
    glen = (offsets[which + 1] - offsets[which])
    st = offsets[which] + (rng.random(n_reads) * (glen - length + 1)).astype(np.int64)
    strands = rng.integers(0, 2, size=n_reads).astype(np.uint8)
    reads = codes[st[:, None] + np.arange(length)[None, :]]
    _substitute(rng, reads, sub)
    rev = strands == 1
    flipped = reads[rev][:, ::-1]
    reads[rev] = np.where(flipped == 4, 4, 3 - flipped)
    ro = np.arange(0, (n_reads + 1) * length, length, dtype=np.int64)
    return reads.reshape(-1).copy(), ro, which.astype(np.int64)


# ---------------------------------------------------------------------------------------
# The five workloads.  Seeds: reference = workload number, reads = 100 + number,
# repeats = 200 + number, absent lookup keys = 304.
# ---------------------------------------------------------------------------------------

def add_gaps(codes, seed, n_runs=0, run_len=(100, 10_000), n_single=0):
    """A copy of codes with ambiguous bases (code 4): n_runs runs of N with uniform lengths
    in run_len (assembly gaps) at uniform starts, plus n_single isolated Ns."""
    rng = np.random.default_rng(seed)
    out = np.array(codes, np.uint8, copy=True)
    if out.size == 0:
        return out
    for _ in range(n_runs):
        L = int(rng.integers(run_len[0], run_len[1] + 1))
        a = int(rng.integers(0, max(out.size - L, 1)))
        out[a:a + L] = 4
    if n_single:
        out[rng.integers(0, out.size, n_single)] = 4
    return out


def to_text(codes, seed=None):
    """Codes as sequence text: A C G T for 0..3 and N for 4; with a seed, a random mix of
    upper and lower case and of other ambiguity letters in place of N."""
    c = np.asarray(codes, np.uint8)
    upper = np.frombuffer(b"ACGTN", np.uint8)[c]
    if seed is None:
        return upper.tobytes()
    rng = np.random.default_rng(seed)
    out = np.where(rng.random(c.size) < 0.5, upper, upper | 0x20).astype(np.uint8)
    amb = np.frombuffer(b"NnRYKMSWBDHV-.*", np.uint8)
    isn = c == 4
    out[isn] = amb[rng.integers(0, amb.size, int(isn.sum()))]
    return out.tobytes()


def workload_tiny():
    """1 Mbp i.i.d. reference; 2,000 x 150 bp reads, both strands, 1 % substitutions;
    pattern '10'; k=15, w=10."""
    ref = random_genome(1_000_000, 1)
    rc, ro, st, sd = fixed_reads(ref, 2000, 150, 101, sub=0.01)
    return dict(name="tiny-1Mbp", ref=ref, ref_offsets=np.array([0, ref.size], np.int64),
                reads=rc, read_offsets=ro, read_start=st, read_strand=sd,
                patterns=["10"], k=15, w=10)


def workload_illumina(ref_len=100_000_000, n_reads=1_000_000):
    """100 Mbp reference with 5 % repeats; 1M x 150 bp reads, 0.5 % substitutions +
    0.05 % 1-bp indels; pattern '10'; k=21, w=11."""
    ref = add_repeats(random_genome(ref_len, 2), 202)
    rc, ro, st, sd = fixed_reads(ref, n_reads, 150, 102, sub=0.005, ins=0.00025, dele=0.00025)
    return dict(name="illumina-100Mbp", ref=ref, ref_offsets=np.array([0, ref.size], np.int64),
                reads=rc, read_offsets=ro, read_start=st, read_strand=sd,
                patterns=["10"], k=21, w=11)


def workload_gapped(ref_len=100_000_000, n_reads=1_000_000):
    """The Illumina-like workload with ambiguous bases: its reference with 50 assembly
    gaps of 20-180 kbp (about 5 % N, the share of N in a human reference assembly) and
    20,000 isolated Ns; its reads with one N call per 1,000 bases on average."""
    d = workload_illumina(ref_len, n_reads)
    d["ref"] = add_gaps(d["ref"], 402, n_runs=50, run_len=(20_000, 180_000), n_single=20_000)
    d["reads"] = add_gaps(d["reads"], 403, n_single=d["reads"].size // 1000)
    d["name"] = "illumina-gapped-100Mbp"
    return d


def workload_fig4(n_pairs=100_000, length=1000, max_rate=0.6, seed=5):
    """Seed-matching experiment: n_pairs sequences of `length` bases cut from an i.i.d.
    genome, each with a copy in which every base is substituted (by one of the three
    other bases) with a per-pair probability drawn uniformly from [0, max_rate], so the
    pairs span the whole range of differences.  Returns (original codes, offsets, copy
    codes, offsets, substitutions per pair)."""
    rng = np.random.default_rng(seed)
    orig = random_genome(n_pairs * length, seed)
    rate = rng.random(n_pairs) * max_rate
    hit = rng.random((n_pairs, length)) < rate[:, None]
    copy = orig.reshape(n_pairs, length).copy()
    n_hit = int(hit.sum())
    copy[hit] = (copy[hit] + rng.integers(1, 4, n_hit, dtype=np.uint8)) % 4
    offs = np.arange(0, (n_pairs + 1) * length, length, dtype=np.int64)
    return orig, offs, copy.reshape(-1), offs.copy(), hit.sum(axis=1).astype(np.int64)


def workload_uneven(ref_len=1_000_000_000, n_short=2_000_000, n_hifi=20_000, n_ont=20_000):
    """1 Gbp reference (same repeat model); one mixed batch of short, HiFi-like and
    ONT-like reads; patterns '10' and '110'; k=21, w=11."""
    ref = add_repeats(random_genome(ref_len, 3), 203)
    short = fixed_reads(ref, n_short, 150, 103, sub=0.005, ins=0.00025, dele=0.00025)
    rng = np.random.default_rng(1103)
    hl = hifi_lengths(n_hifi, rng)
    ol = ont_lengths(n_ont, rng)
    hifi = variable_reads(ref, hl, 2103, 0.005, 0.0025, 0.0025)
    ont = variable_reads(ref, ol, 3103, 0.04, 0.02, 0.02)
    codes, offs = concat([short, hifi, ont])
    return dict(name="uneven-1Gbp", ref=ref, ref_offsets=np.array([0, ref.size], np.int64),
                reads=codes, read_offsets=offs,
                classes=dict(short=(0, n_short), hifi=(n_short, n_short + n_hifi),
                             ont=(n_short + n_hifi, n_short + n_hifi + n_ont)),
                patterns=["10", "110"], k=21, w=11)


def absent_keys(n, seed=304):
    """Random 64-bit lookup keys (the caller removes any that happen to be present)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2**64, size=n, dtype=np.uint64)


def workload_containment(n_genomes=1000, n_reads=10_000_000, n_source=50):
    """1,000 genomes of 1-5 Mbp (30 % share a 10 % block with a partner at 5 %
    divergence); 10M x 150 bp reads from 50 genomes with lognormal(0, 1) abundances and
    1 % substitutions; pattern '10'; k=21, w=11."""
    codes, offs = genome_db(n_genomes, 5)
    rc, ro, src = sample_from_genomes(codes, offs, n_reads, n_source, 150, 105, sub=0.01)
    return dict(name="containment-1000", ref=codes, ref_offsets=offs, reads=rc,
                read_offsets=ro, read_source=src, patterns=["10"], k=21, w=11)
