"""CPU oracle for the sparse, truncated state vector: TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may
import anything here. The product package never does, and the two share no
code. Modules:

  dict_oracle - plain-Python dictionary-of-terms simulator (small cases)
  c_oracle    - the same semantics in plain C (larger cases, timed baseline)
  dense       - textbook dense 2^n simulator used only to pin the oracle
"""
