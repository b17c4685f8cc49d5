"""Test-only FP64 oracle (C) and exact-rational checker.  Never imported by the product package."""
