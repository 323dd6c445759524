"""Test-only CPU oracle for the sparse permanent (see oracle.py)."""
