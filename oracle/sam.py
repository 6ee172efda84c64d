"""Oracle of the mapping-quality filter and SAM records (test
infrastructure: only tests, the smoke check and the benchmark's CPU
baseline use it).

Follows the Methods paragraph on mapping qualities, read lengths, SAM
output and source code: the MAPQ field is -100 log2 p, where p, the
probability that the alignment is wrong, is taken as the ratio of the
second-best to the best fragment score; a read counts as mapped when that
ratio is below 0.9 (the first-phase paragraph), i.e. when its mapping
quality exceeds -100 log2 0.9 = 15.2.  The Results raise the threshold to 62
for the ancient-DNA reads.

Readings (the paper does not fix them):
  - the MAPQ field is the integer part of -100 log2(s2/s1), capped at 254
    (SAM reserves 255 for "unavailable"); s2 <= 0 or no second fragment
    gives the cap; s1 <= 0 gives 0 and the read is unmapped;
  - a read is mapped when s1 > 0, s2 * den < s1 * num (the ratio rule,
    9/10 by default) and MAPQ > min_mapq (the integer threshold, off by
    default);
  - records follow SAM v1: QNAME FLAG RNAME POS MAPQ CIGAR RNEXT PNEXT TLEN
    SEQ QUAL, tab-separated, then the tag AS:i (the NW score) for mapped
    reads.  FLAG 16 marks the reverse strand; SEQ is the read on the
    forward genome strand (reverse-complemented for strand 1); QUAL is the
    read's Phred+33 string in SEQ's order (reversed for strand 1), or "*"
    for a read without qualities.  An unmapped read has FLAG 4, RNAME "*",
    POS 0, MAPQ 0, CIGAR "*", SEQ and QUAL as given; a read marked invalid
    by the scan has SEQ and QUAL "*".  A truncated CIGAR is written as "*".
"""
from __future__ import annotations

import math

MAPQ_CAP = 254
INVALID = -2  # frag[0] of a read the scan marked invalid

_COMP = {ord("A"): "T", ord("C"): "G", ord("G"): "C", ord("T"): "A", ord("N"): "N"}


def mapq(s1: int, s2: int) -> int:
    """Integer MAPQ of a read with best score s1 and second-best s2 (s2 < 0
    when there is no second fragment)."""
    if s1 <= 0:
        return 0
    if s2 <= 0:
        return MAPQ_CAP
    q = math.floor(-100.0 * math.log2(s2 / s1))
    return max(0, min(MAPQ_CAP, q))


def is_mapped(s1: int, s2: int, num: int = 9, den: int = 10, min_mapq: int = -1) -> bool:
    return s1 > 0 and max(s2, 0) * den < s1 * num and mapq(s1, s2) > min_mapq


def revcomp(read: bytes) -> str:
    return "".join(_COMP[c] for c in reversed(read.upper()))


def header(rname: str, G: int) -> str:
    return "@HD\tVN:1.6\tSO:unsorted\n@SQ\tSN:%s\tLN:%d\n@PG\tID:maxss\tPN:maxss\n" % (rname, G)


def record(name: str, read: bytes, top, aln: dict | None, rname: str, num: int = 9,
           den: int = 10, min_mapq: int = -1, truncated: bool = False,
           qual: bytes | None = None) -> str:
    """One SAM line (with its newline) from the oracle's own results: `top`
    the read's top-2 record (oracle.scan), `aln` the dict of oracle.align_one
    (score, strand, ref_begin, ref_end, cigar); `truncated` writes CIGAR "*";
    `qual` the read's Phred+33 qualities as given (None: QUAL "*")."""
    f1 = int(top["frag"][0])
    s1 = int(top["score"][0])
    s2 = int(top["score"][1]) if int(top["frag"][1]) >= 0 else -1
    if f1 == INVALID:
        return "\t".join([name, "4", "*", "0", "0", "*", "*", "0", "0", "*", "*"]) + "\n"
    if not is_mapped(s1, s2, num, den, min_mapq):
        q = qual.decode() if qual else "*"
        return "\t".join([name, "4", "*", "0", "0", "*", "*", "0", "0", read.decode().upper(),
                          q]) + "\n"
    strand = int(aln["strand"])
    seq = read.decode().upper() if strand == 0 else revcomp(read)
    q = "*" if not qual else (qual.decode() if strand == 0 else qual.decode()[::-1])
    fields = [name, "16" if strand else "0", rname, str(int(aln["ref_begin"]) + 1),
              str(mapq(s1, s2)), "*" if truncated else aln["cigar"], "*", "0", "0", seq, q,
              "AS:i:%d" % int(aln["score"])]
    return "\t".join(fields) + "\n"
