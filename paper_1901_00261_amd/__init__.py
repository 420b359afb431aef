"""Compact 6th/8th-order gas-kinetic scheme on MI355X (HIP library + Python binding)."""
