"""CPU oracles for the counting quotient filter.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import, call, link or execute anything in this package.
The GPU library never does, and the two share no code.

  oqf.c / oqf.py : plain sequential CQF (decode, modify, re-emit a cluster).
  brute.py       : the canonical table computed directly from the multiset.
"""
