"""ORACLE -- test infrastructure (plain FP64 CPU tracker); not part of the product."""
