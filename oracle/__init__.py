"""CPU oracle for the assembly-free theta-scheme heat solver (test infrastructure only)."""
