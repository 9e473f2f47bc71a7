"""FP64 CPU oracle for the Shan-Chen lattice Boltzmann hot path.

TEST INFRASTRUCTURE: imported only by tests/, __graft_entry__.smoke() and the
CPU-baseline leg of bench.py.  Shares no code with the GPU library.

Parity pins live in tests/ (test_tables.py, test_oracle_*.py).
"""
