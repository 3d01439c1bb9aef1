"""Batched Wiener-filter MAP and band-power estimation on MI355X (binding placeholder)."""
