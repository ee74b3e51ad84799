"""Test-only FP64 reference implementations of LSG-CPD (see lsgcpd_oracle)."""
