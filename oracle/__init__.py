"""FP64 CPU oracle for the SCD estimators (FAM and SSCA).

TEST INFRASTRUCTURE ONLY: this package exists to check the GPU library. Only ``tests/``,
``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg may import it. The GPU library
(``paper_2506_18003_amd``) never imports it, and the two share no code.

Modules:
  scd_oracle  vectorised numpy FP64 definitions (channelizer Eq. 3, SSCA Eq. 6-7, SSCA_2DFFT Eq. 10-16,
              FAM Eq. 4-5, coordinate maps)
  brute       pure-Python direct sums of Eq. (1)-(3) and (5) used to pin ``scd_oracle`` on tiny inputs
"""
