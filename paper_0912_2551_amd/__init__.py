"""On-the-fly statistical model checking of mass-action reaction networks on MI355X."""
