"""Mutation check of the oracle's pins (CPU only; not collected by pytest).

Each entry plants one plausible mistake in a copy of oracle/godiet_oracle.c, builds the
copy in a temporary directory, and runs tests/test_oracle.py against it (the oracle
package loads the copy through GODIET_ORACLE_LIB).  Every mutant must make at least one
pin fail; the script prints one line per mutant and exits 1 if any survives.  The tree's
own oracle source and library are never modified.

    python tests/oracle_mutants.py
"""
import os
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "godiet_oracle.c")

# (what the mistake is, text in the oracle, replacement)
MUTANTS = [
    ("strand sign", "strand[i] = rc < fwd ? 1 : 0;", "strand[i] = rc > fwd ? 1 : 0;"),
    ("reverse-complement index",
     "(3 - PS[i + (uint64_t)k - 1 - t])", "(3 - PS[i + (uint64_t)k - 1 - t + (t==0)])"),
    ("hash shift constant", "z = (z ^ (z >> 27))", "z = (z ^ (z >> 28))"),
    ("window range of a k-mer",
     "uint64_t s_lo = i + 1 >= (uint64_t)w ? i + 1 - (uint64_t)w : 0;",
     "uint64_t s_lo = i >= (uint64_t)w ? i - (uint64_t)w + 2 : 0;"),
    ("pattern phase sign",
     "uint64_t t = (j % p + p - (a % p)) % p;", "uint64_t t = (j % p + (a % p)) % p;"),
    ("patterned instead of original coordinates",
     "vals[out] = (orig[i] << 1) | strand[i];", "vals[out] = ((uint64_t)i << 1) | strand[i];"),
    ("alignment tie rule",
     "if (score > best_score) { best_score = score; best = s; }",
     "if (score >= best_score && score > 0) { best_score = score; best = s; }"),
    ("frequency filter bound",
     "if (max_occ > 0 && ub - lb >= max_occ) continue;",
     "if (max_occ > 0 && ub - lb > max_occ) continue;"),
    ("alignment limit t",
     "if (t > 0 && (uint64_t)t < nstar) nstar = t;",
     "if (t > 1 && (uint64_t)t < nstar) nstar = t;"),
    ("sequence-id field of 64-bit values",
     "else r[i].val = ((uint64_t)s << 32) | (pos << 1) | strand;",
     "else r[i].val = ((uint64_t)s << 31) | (pos << 1) | strand;"),
    ("window maximum instead of minimum",
     "if (!wany[s] || h[t] < wmin[s]) wmin[s] = h[t];",
     "if (!wany[s] || h[t] > wmin[s]) wmin[s] = h[t];"),
    ("palindromes not excluded",
     "if (fwd == rc) { ok[i] = 0; h[i] = 0; strand[i] = 0; continue; }",
     "if (0) { ok[i] = 0; h[i] = 0; strand[i] = 0; continue; }"),
    ("anchor strand without the index strand",
     "anchors[4 * n + 3] = (uint32_t)((mv[j] ^ ivals[e]) & 1);",
     "anchors[4 * n + 3] = (uint32_t)(mv[j] & 1);"),
    ("reverse-strand location as a diagonal",
     "list[i].loc = a[3] ? (int64_t)a[2] + (int64_t)a[1] : (int64_t)a[2] - (int64_t)a[1];",
     "list[i].loc = (int64_t)a[2] - (int64_t)a[1];"),
    ("voting distance exclusive",
     "list[j].loc <= c.loc + (int64_t)D) j++;", "list[j].loc < c.loc + (int64_t)D) j++;"),
    ("vote threshold strict", "if (c.votes >= V) win[nw++] = c;", "if (c.votes > V) win[nw++] = c;"),
    ("rescue keeps the last best", "if (c.votes > rescue.votes) rescue = c;",
     "if (c.votes >= rescue.votes) rescue = c;"),
    ("winners by ascending votes", "if (a->votes != b->votes) return a->votes > b->votes ? -1 : 1;",
     "if (a->votes != b->votes) return a->votes < b->votes ? -1 : 1;"),
    ("Wang hash multiplier", "key = (key * 265u) & mask;", "key = (key * 273u) & mask;"),
    ("Wang hash first step unmasked", "key = (~key + (key << 21)) & mask;",
     "key = (~key + (key << 21));"),
    ("N does not end a run", "if (i < n && PS[i] != 4) continue;", "if (i < n) continue;"),
    ("run restarts at the N instead of after it", "        r0 = i + 1;", "        r0 = i;"),
    ("edit distance: free substitutions", "uint64_t d = prev[j - 1] + (a[i - 1] != b[j - 1] ? 1 : 0);",
     "uint64_t d = prev[j - 1];"),
    ("spaced-seed mask off by one", "if (alg == 0 || P->bit[j % P->p]) buf[n++]",
     "if (alg == 0 || P->bit[(j + 1) % P->p]) buf[n++]"),
    ("minimizers sketched with the pattern", "alg == 1 ? &one : P", "P"),
    ("accepted pairs need a strictly higher rate", "if (m * tt >= tm * t) c++;",
     "if (m * tt > tm * t) c++;"),
    ("containment counts every genome hash",
     "if (bsearch(&gh[i].val, sample, (size_t)nu, sizeof(uint64_t), u64_cmp)) counts[g]++;",
     "if (1) counts[g]++;"),
]


def main():
    src = open(SRC).read()
    survived = 0
    with tempfile.TemporaryDirectory() as tmp:
        for i, (what, old, new) in enumerate(MUTANTS):
            if src.count(old) != 1:
                print("[%s] target text not found once in the oracle" % what)
                survived += 1
                continue
            c = os.path.join(tmp, "m%d.c" % i)
            so = os.path.join(tmp, "m%d.so" % i)
            with open(c, "w") as f:
                f.write(src.replace(old, new))
            subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", so, c])
            env = dict(os.environ, GODIET_ORACLE_LIB=so)
            try:
                r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p",
                                    "no:cacheprovider",
                                    os.path.join(ROOT, "tests", "test_oracle.py")],
                                   cwd=ROOT, env=env, capture_output=True, text=True,
                                   timeout=120)
                last = (r.stdout.strip().splitlines() or ["?"])[-1]
                killed = r.returncode != 0
            except subprocess.TimeoutExpired:     # a mutant that never ends fails too
                last, killed = "timed out", True
            survived += 0 if killed else 1
            print("%-8s %-45s %s" % ("killed" if killed else "SURVIVED", what, last))
    print("%d of %d mutants killed" % (len(MUTANTS) - survived, len(MUTANTS)))
    return 1 if survived else 0


if __name__ == "__main__":
    sys.exit(main())
