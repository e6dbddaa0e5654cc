"""CPU oracles for the counting quotient filter and the two-choice filter.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import, call, link or execute anything in this package.
The GPU library never does, and the two share no code.

  oqf.c / oqf.py : plain sequential CQF (decode, modify, re-emit a cluster).
  brute.py       : the canonical table computed directly from the multiset.
  tcf.py         : the two-choice filter (point rules one key at a time, the
                   bulk rules batch by batch, a validity check of tables that
                   concurrent point inserts built).
"""
